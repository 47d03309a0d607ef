// Conservative binning (vsr_bin): per 8x8 tile, the triangles that may
// cover one of its pixels, in depth-bucket order.
//
// Two workgroup shapes share the gathering code (gather.hpp):
//   bin_block  one 256-thread workgroup per 32x32 block (4x4 tiles, wave w
//              owns the 2x2 tiles of quadrant w).  The block cap gathers the
//              candidates once; each survivor is tested against the four
//              quadrant (super-tile) caps and then the tiles of the
//              quadrants it may meet; survivors go straight to the output
//              lists, which each wave sorts in place at the end.  For list
//              capacities up to 256.
//   bin_super  one 256-thread workgroup per 16x16 super-tile (2x2 tiles,
//              wave w owns tile w), for deep lists.
// bin_super appends survivors to LDS lists and each wave writes its tile's
// list with a counting sort by depth bucket.
//
// With 16x16 bin tiles (BinArgs::tile16) there is one list per super-tile:
// the survivors that may meet the super-tile (its cap and edge planes,
// quad_may_see), appended to LDS and written once, in depth-bucket order.
// The rasterizer then keeps, for each 8x8 tile, the entries that pass the
// 8x8 binner's own tile test, so each tile sees exactly that binner's list.
#pragma once
#include "gather.hpp"

namespace vsr {

struct BinArgs {
    const void* map;
    int64_t ntiles;
    int32_t fmt, depth, lds_cap, all;
    int32_t ntx, nty;
    int32_t tile16, pad;  // tile16: one list per 16x16 super-tile instead of per 8x8 tile
    const void* setup;
    int64_t n;
    void* bins;
    uint32_t* status;  // overflowed-tile counter
    Rot rot;           // camera -> world

    __device__ inline void globalize() {
        map = to_global(map);
        setup = to_global(setup);
        bins = to_global(bins);
        status = to_global(status);
    }
};

__device__ inline void bin_super(const BinArgs& A0, int64_t sidx) {
    BinArgs A = A0;
    A.globalize();
    extern __shared__ uint32_t lists[];  // kSupTiles x lds_cap
    __shared__ SuperShared sh;
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    int64_t tile;
    int tx, ty;
    const bool present = super_tile_of(sidx, w, A.ntx, A.nty, tile, tx, ty);
    super_setup(sh, map_caps(A.map, A.ntiles, A.fmt), map_sups(A.map, A.ntiles, A.fmt), A.rot,
                scene_view(A.setup, A.n).face_count, present, tile, sidx);
    const bool any = sh.sup[1].z != 0.0f;
    const SceneView S = scene_view(A.setup, A.n);
    const uint32_t lcap = uint32_t(A.lds_cap);
    uint32_t live_mask = 0;
#pragma unroll
    for (int q = 0; q < kSupTiles; ++q)
        if (sh.cap[q][1].z != kCapEmpty) live_mask |= 1u << q;

    auto append = [&](uint32_t mask, uint32_t rank) {
#pragma unroll
        for (int q = 0; q < kSupTiles; ++q) {
            if (mask & (1u << q)) {
                uint32_t pos = atomicAdd(&sh.cnt[q], 1u);
                if (pos < lcap) lists[q * lcap + pos] = rank;
            }
        }
    };
    if (any && A.all) {
        for (int64_t k0 = 0; k0 < A.n; k0 += 256) {
            int64_t r = k0 + tid;
            if (r < A.n && S.cap[2 * r + 1].z != kCapEmpty) append(live_mask, uint32_t(r));
        }
    } else if (any) {
        auto visit = [&](bool valid, float4 a, float ch_t, float3 n0, float3 n1, float3 n2, uint32_t rank) {
            uint32_t mask = 0;
            // the tile caps are read from LDS here rather than held in 32
            // registers across the gathering loop
            asm volatile("" ::: "memory");
            if (valid) {
#pragma unroll
                for (int q = 0; q < kSupTiles; ++q)
                    if ((live_mask >> q) & 1u)
                        if (sub_may_see(sh.cap[q][0], sh.cap[q][1], a, ch_t, n0, n1, n2)) mask |= 1u << q;
            }
            if (mask) append(mask, rank);
        };
        gather_slices(sh, S, 0, kSlices, [&](const uint32_t* chunk, uint32_t n) {
            const bool valid = uint32_t(threadIdx.x) < n;
            visit_record(S, valid, valid ? chunk[threadIdx.x] : 0u, visit);
        }, [] {});
    }
    __syncthreads();

    const uint32_t cnt = sh.cnt[w];
    const bool keep = present && cnt <= uint32_t(A.depth);
    char* bb = reinterpret_cast<char*>(A.bins);
    if (keep) {
        uint32_t* out = reinterpret_cast<uint32_t*>(bb + 256 + align256(A.ntiles * 4)) + tile * A.depth;
        bucket_sort_wave(lists + w * lcap, cnt, sh.bk[w], bucket_shift(A.n), out);
    }
    if (present && lane == 0) {
        reinterpret_cast<uint32_t*>(bb + 256)[tile] = cnt;
        if (!keep) atomicAdd(A.status, 1u);
    }
}

__global__ __launch_bounds__(256) void k_bin(BinArgs A) {
    const int64_t nsx = (A.ntx + 1) / 2;  // super-tiles per row
    bin_super(A, band_remap(blockIdx.x, gridDim.x, max(int64_t(1), nsx * kBandPx / (2 * kTile))));
}

// quad_may_see is defined with the 32x32 blocks below.
__device__ inline bool quad_may_see(float4 s0, float4 s1, float4 a, float ch_t, float3 n0, float3 n1, float3 n2);

// One 16x16 bin tile per workgroup: the gather survivors that may meet the
// super-tile go to one LDS list, which wave 0 writes in depth-bucket order.
__device__ inline void bin_super16(const BinArgs& A0, int64_t sidx) {
    BinArgs A = A0;
    A.globalize();
    extern __shared__ uint32_t lists[];  // lds_cap
    __shared__ SuperShared sh;
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    int64_t tile;
    int tx, ty;
    const bool present = super_tile_of(sidx, w, A.ntx, A.nty, tile, tx, ty);
    super_setup(sh, map_caps(A.map, A.ntiles, A.fmt), map_sups(A.map, A.ntiles, A.fmt), A.rot,
                scene_view(A.setup, A.n).face_count, present, tile, sidx);
    const bool any = sh.sup[1].z != 0.0f;
    const SceneView S = scene_view(A.setup, A.n);
    const uint32_t lcap = uint32_t(A.lds_cap);
    auto append = [&](uint32_t rank) {
        const uint32_t pos = atomicAdd(&sh.cnt[0], 1u);
        if (pos < lcap) lists[pos] = rank;
    };
    if (any && A.all) {
        for (int64_t k0 = 0; k0 < A.n; k0 += 256) {
            int64_t r = k0 + tid;
            if (r < A.n && S.cap[2 * r + 1].z != kCapEmpty) append(uint32_t(r));
        }
    } else if (any) {
        const float4 s0 = sh.sup[0], s1 = sh.sup[1];
        gather_slices(sh, S, 0, kSlices, [&](const uint32_t* chunk, uint32_t n) {
            const bool valid = uint32_t(threadIdx.x) < n;
            visit_record(S, valid, valid ? chunk[threadIdx.x] : 0u,
                         [&](bool v, float4 a, float ch_t, float3 n0, float3 n1, float3 n2, uint32_t rank) {
                             if (v && quad_may_see(s0, s1, a, ch_t, n0, n1, n2)) append(rank);
                         });
        }, [] {});
    }
    __syncthreads();
    if (w == 0) {
        const uint32_t cnt = sh.cnt[0];
        const bool keep = cnt <= uint32_t(A.depth);
        char* bb = reinterpret_cast<char*>(A.bins);
        uint32_t* out = reinterpret_cast<uint32_t*>(bb + 256 + align256(A.ntiles * 4)) + sidx * A.depth;
        if (keep) bucket_sort_wave(lists, cnt, sh.bk[0], bucket_shift(A.n), out);
        if (lane == 0) {
            reinterpret_cast<uint32_t*>(bb + 256)[sidx] = cnt;
            if (!keep) atomicAdd(A.status, 1u);
        }
    }
}

__global__ __launch_bounds__(256) void k_bin16(BinArgs A) {
    const int64_t nsx = (A.ntx + 1) / 2;
    bin_super16(A, band_remap(blockIdx.x, gridDim.x, max(int64_t(1), nsx * kBandPx / (2 * kTile))));
}

// ------------------------------------------------ 32x32 blocks ----------

constexpr int kBlkTiles = 16;
constexpr uint32_t kQueue = 320;  // >= 63 carried + 256 of one chunk

struct BlockShared {
    SuperShared g;                // gathering state; g.sup = block cap
    float4 tcap[kBlkTiles][2];    // tile caps, tile 4q + (2 dy + dx) of quadrant q
    float4 qcap[4][2];            // quadrant (super-tile) caps, super-tile layout
    uint32_t tcnt[kBlkTiles];
    uint32_t ttile[kBlkTiles];    // map tile of each slot (its output list)
    uint32_t qn[4];               // survivors filed for quadrant q and not yet tested ...
    uint32_t ql[4][kQueue];       // ... and their cell-ordered positions
};

// Tile (tx, ty) of slot t (quadrant t >> 2) of block b; false outside the map.
__device__ inline bool block_tile_of(int64_t b, int t, int ntx, int nty, int64_t& tile) {
    const int nbx = (ntx + 3) / 4;
    const int bx = int(b % nbx), by = int(b / nbx);
    const int q = t >> 2, d = t & 3;
    const int tx = 4 * bx + 2 * (q & 1) + (d & 1), ty = 4 * by + 2 * (q >> 1) + (d >> 1);
    tile = int64_t(ty) * ntx + tx;
    return tx < ntx && ty < nty;
}

// May a triangle meet a pixel of the super-tile with cap (s0, s1) (super-tile
// layout)?  Same conservative tests as sub_may_see.
// Without branches, as sub_may_see.
__device__ inline bool quad_may_see(float4 s0, float4 s1, float4 a, float ch_t, float3 n0, float3 n1, float3 n2) {
    const float dx = s0.x - a.x, dy = s0.y - a.y, dz = s0.z - a.z;
    const float chord2 = dx * dx + dy * dy + dz * dz;
    const float sm = s0.w * ch_t + s1.y * a.w;
    const bool apart = (a.w < kBinWide) & (chord2 > 4.0f * sm * sm * (1.0f + 1e-6f) + 1e-12f);
    const float3 c = f3(s0.x, s0.y, s0.z);
    const float lim = -2.0f * s1.x * s1.y - 1e-6f;  // -sin(rho)
    const float d0 = dot3(n0, c), d1 = dot3(n1, c), d2 = dot3(n2, c);
    const bool outside = (d0 < lim) | (d1 < lim) | (d2 < lim);
    // s1.z == 0: no pixel with a direction; s1.w != 0: wide
    return (s1.z != 0.0f) & ((s1.w != 0.0f) | !(apart | outside));
}

// In-place counting sort of one wave's list of cnt <= 256 ranks (global
// memory written by this workgroup) by depth bucket: the wave holds the list
// in registers while it counts, then scatters it back.
__device__ inline void bucket_sort_inplace(uint32_t* list, uint32_t cnt_any, uint32_t* bk, int shift) {
    const int lane = threadIdx.x & 63;
    const uint32_t cnt = __builtin_amdgcn_readfirstlane(cnt_any);
    if (cnt < 2) return;
    uint32_t v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint32_t i = uint32_t(lane + 64 * k);
        v[k] = 0u;
        if (64u * k < cnt && i < cnt) v[k] = list[i];
    }
    reinterpret_cast<uint4*>(bk)[lane] = make_uint4(0u, 0u, 0u, 0u);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (64u * k < cnt && uint32_t(lane + 64 * k) < cnt) atomicAdd(&bk[v[k] >> shift], 1u);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const uint4 c4 = reinterpret_cast<const uint4*>(bk)[lane];
    const uint32_t run = c4.x + c4.y + c4.z + c4.w;
    uint32_t x = run;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    const uint32_t base = x - run;
    __builtin_amdgcn_wave_barrier();
    reinterpret_cast<uint4*>(bk)[lane] = make_uint4(base, base + c4.x, base + c4.x + c4.y, base + c4.x + c4.y + c4.z);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (64u * k < cnt && uint32_t(lane + 64 * k) < cnt) list[atomicAdd(&bk[v[k] >> shift], 1u)] = v[k];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// The block shape needs list capacity <= 256 (see use_blocks).  Survivors
// go straight to their tile's slots of the output lists (the first `depth`
// appended; a tile with more is reported as overflowed), and each wave
// sorts its tiles' lists in place at the end, so the workgroup's LDS holds
// no lists: more workgroups fit on a CU.
__device__ inline void bin_block(const BinArgs& A0, int64_t b) {
    BinArgs A = A0;
    A.globalize();
    __shared__ BlockShared sh;
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const SceneView S = scene_view(A.setup, A.n);
    const uint32_t depth = uint32_t(A.depth);
    char* bb = reinterpret_cast<char*>(A.bins);
    uint32_t* const out = reinterpret_cast<uint32_t*>(bb + 256 + align256(A.ntiles * 4));
    const int nsx = (A.ntx + 1) / 2, nsy = (A.nty + 1) / 2, nbx = (A.ntx + 3) / 4;
    if (tid < kBlkTiles) {
        int64_t tile;
        float4 c0 = empty_cap0(), c1 = empty_cap1();
        if (block_tile_of(b, tid, A.ntx, A.nty, tile)) load_tile_cap(map_caps(A.map, A.ntiles, A.fmt), tile, A.rot, c0, c1);
        sh.tcap[tid][0] = c0;
        sh.tcap[tid][1] = c1;
        sh.tcnt[tid] = 0;
        sh.ttile[tid] = uint32_t(tile);  // only used for tiles inside the map
    } else if (tid < kBlkTiles + 4) {
        const int q = tid - kBlkTiles;
        const int sx = 2 * int(b % nbx) + (q & 1), sy = 2 * int(b / nbx) + (q >> 1);
        float4 s0 = make_float4(0.f, 0.f, 1.f, 1.f), s1 = make_float4(1.f, 0.f, 0.f, 0.f);  // no pixel
        if (sx < nsx && sy < nsy) load_tile_cap(map_sups(A.map, A.ntiles, A.fmt), int64_t(sy) * nsx + sx, A.rot, s0, s1);
        sh.qcap[q][0] = s0;
        sh.qcap[q][1] = s1;
    } else if (tid == kBlkTiles + 4) {
        float4 s0, s1;
        load_tile_cap(map_blks(A.map, A.ntiles, A.fmt, A.ntx, A.nty), b, A.rot, s0, s1);
        sh.g.sup[0] = s0;
        sh.g.sup[1] = s1;
    }
    for (int q = tid; q < kSlices * 64; q += 256) sh.g.fc[q] = S.face_count[q];
    __syncthreads();
    setup_rects(sh.g);
    const bool any = sh.g.sup[1].z != 0.0f;

    auto append = [&](uint32_t mask, uint32_t rank) {
        while (mask) {
            const int t = __ffs(mask) - 1;
            mask &= mask - 1;
            const uint32_t pos = atomicAdd(&sh.tcnt[t], 1u);
            if (pos < depth) out[int64_t(sh.ttile[t]) * depth + pos] = rank;
        }
    };
    if (any && A.all) {
        uint32_t live = 0;
        for (int t = 0; t < kBlkTiles; ++t)
            if (sh.tcap[t][1].z != kCapEmpty) live |= 1u << t;
        for (int64_t k0 = 0; k0 < A.n; k0 += 256) {
            int64_t r = k0 + tid;
            if (r < A.n && S.cap[2 * r + 1].z != kCapEmpty) append(live, uint32_t(r));
        }
    } else if (any) {
        // Each chunk of survivors: every thread tests one survivor against
        // the four quadrant caps and files it in the queues of the quadrants
        // it may meet; then wave w tests the whole waves (64 entries) of
        // quadrant w's queue against its four tiles and moves the rest to
        // the front, for the next chunk; what is left is tested at the end.
        // A wave owns its tiles' counters, so it appends with ballots.
        if (tid < 4) sh.qn[tid] = 0;
        __syncthreads();
        auto drain = [&](bool all) {
            const uint32_t nq = __builtin_amdgcn_readfirstlane(sh.qn[w]);
            const uint32_t m = all ? nq : nq & ~63u;
            if (m == 0) return;
            uint32_t tn[4];   // the wave's tile counts, kept identical in every lane
            uint32_t* tl[4];  // and their output lists
#pragma unroll
            for (int d = 0; d < 4; ++d) {
                tn[d] = __builtin_amdgcn_readfirstlane(sh.tcnt[4 * w + d]);
                tl[d] = out + int64_t(uint32_t(__builtin_amdgcn_readfirstlane(sh.ttile[4 * w + d]))) * depth;
            }
            for (uint32_t i0 = 0; i0 < m; i0 += 64) {
                // the tile caps are read from LDS where they are used rather
                // than held in 32 registers across the loop
                asm volatile("" ::: "memory");
                const bool v = i0 + uint32_t(lane) < m;
                visit_record(S, v, v ? sh.ql[w][i0 + uint32_t(lane)] : 0u,
                             [&](bool valid, float4 a, float ch_t, float3 n0, float3 n1, float3 n2, uint32_t rank) {
#pragma unroll
                                 for (int d = 0; d < 4; ++d) {
                                     const bool on = valid && sub_may_see(sh.tcap[4 * w + d][0], sh.tcap[4 * w + d][1],
                                                                          a, ch_t, n0, n1, n2);
                                     const uint64_t bal = __ballot(on);
                                     const uint32_t pos = tn[d] + __builtin_amdgcn_mbcnt_hi(
                                                                      uint32_t(bal >> 32),
                                                                      __builtin_amdgcn_mbcnt_lo(uint32_t(bal), 0u));
                                     if (on && pos < depth) tl[d][pos] = rank;
                                     tn[d] += uint32_t(__popcll(bal));
                                 }
                             });
            }
            // fewer than 64 left (none at the end): to the front of the queue
            const uint32_t left = nq - m;
            const uint32_t keep = uint32_t(lane) < left ? sh.ql[w][m + uint32_t(lane)] : 0u;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            if (uint32_t(lane) < left) sh.ql[w][lane] = keep;
            if (lane == 0) {
#pragma unroll
                for (int d = 0; d < 4; ++d) sh.tcnt[4 * w + d] = tn[d];
                sh.qn[w] = left;  // appended to after the next barrier
            }
        };
        auto visit_chunk = [&](const uint32_t* chunk, uint32_t n) {
            if (uint32_t(tid) < n) {
                const uint32_t p = chunk[tid];
                visit_record(S, true, p, [&](bool, float4 a, float ch_t, float3 n0, float3 n1, float3 n2, uint32_t) {
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        if (quad_may_see(sh.qcap[q][0], sh.qcap[q][1], a, ch_t, n0, n1, n2))
                            sh.ql[q][atomicAdd(&sh.qn[q], 1u)] = p;
                });
            }
            __syncthreads();
            drain(false);
            __syncthreads();
        };
        gather_slices(sh.g, S, 0, kSlices, visit_chunk, [] {});
        drain(true);
    }
    __syncthreads();

    // wave w sorts the lists of quadrant w's tiles
    const int shift = bucket_shift(A.n);
    for (int d = 0; d < 4; ++d) {
        const int t = 4 * w + d;
        int64_t tile;
        if (!block_tile_of(b, t, A.ntx, A.nty, tile)) continue;
        const uint32_t cnt = sh.tcnt[t];
        const bool keep = cnt <= depth;
        if (keep) bucket_sort_inplace(out + tile * depth, cnt, sh.g.bk[w], shift);
        if (lane == 0) {
            reinterpret_cast<uint32_t*>(bb + 256)[tile] = cnt;
            if (!keep) atomicAdd(A.status, 1u);
        }
    }
}

__global__ __launch_bounds__(256) void k_bin_block(BinArgs A) { bin_block(A, xcd_remap(blockIdx.x, gridDim.x)); }

struct Block16Shared {
    SuperShared g;                // gathering state; g.sup = block cap
    float4 qcap[4][2];            // quadrant (super-tile) caps, super-tile layout
    uint32_t qn[4];               // entries appended to quadrant q's list
};

// 16x16 bin tiles from 32x32 blocks: the block cap gathers the candidates
// once; every survivor is tested against the four quadrant (super-tile)
// caps and appended to the LDS list of each quadrant it may meet; at the
// end wave w writes quadrant w's list once, in depth-bucket order.
__device__ inline void bin_block16(const BinArgs& A0, int64_t b) {
    BinArgs A = A0;
    A.globalize();
    extern __shared__ uint32_t qlist[];  // 4 x lds_cap
    __shared__ Block16Shared sh;
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const SceneView S = scene_view(A.setup, A.n);
    const uint32_t lcap = uint32_t(A.lds_cap);
    const int nsx = (A.ntx + 1) / 2, nsy = (A.nty + 1) / 2, nbx = (A.ntx + 3) / 4;
    if (tid < 4) {
        const int q = tid;
        const int sx = 2 * int(b % nbx) + (q & 1), sy = 2 * int(b / nbx) + (q >> 1);
        float4 s0 = make_float4(0.f, 0.f, 1.f, 1.f), s1 = make_float4(1.f, 0.f, 0.f, 0.f);  // no pixel
        if (sx < nsx && sy < nsy) load_tile_cap(map_sups(A.map, A.ntiles, A.fmt), int64_t(sy) * nsx + sx, A.rot, s0, s1);
        sh.qcap[q][0] = s0;
        sh.qcap[q][1] = s1;
        sh.qn[q] = 0;
    } else if (tid == 4) {
        float4 s0, s1;
        load_tile_cap(map_blks(A.map, A.ntiles, A.fmt, A.ntx, A.nty), b, A.rot, s0, s1);
        sh.g.sup[0] = s0;
        sh.g.sup[1] = s1;
    }
    for (int q = tid; q < kSlices * 64; q += 256) sh.g.fc[q] = S.face_count[q];
    __syncthreads();
    setup_rects(sh.g);
    const bool any = sh.g.sup[1].z != 0.0f;
    auto append = [&](int q, uint32_t rank) {
        const uint32_t pos = atomicAdd(&sh.qn[q], 1u);
        if (pos < lcap) qlist[q * lcap + pos] = rank;
    };
    if (any && A.all) {
        for (int64_t k0 = 0; k0 < A.n; k0 += 256) {
            int64_t r = k0 + tid;
            if (r < A.n && S.cap[2 * r + 1].z != kCapEmpty)
                for (int q = 0; q < 4; ++q)
                    if (sh.qcap[q][1].z != 0.0f) append(q, uint32_t(r));
        }
    } else if (any) {
        gather_slices(sh.g, S, 0, kSlices, [&](const uint32_t* chunk, uint32_t n) {
            if (uint32_t(tid) < n) {
                visit_record(S, true, chunk[tid],
                             [&](bool, float4 a, float ch_t, float3 n0, float3 n1, float3 n2, uint32_t rank) {
#pragma unroll
                                 for (int q = 0; q < 4; ++q)
                                     if (quad_may_see(sh.qcap[q][0], sh.qcap[q][1], a, ch_t, n0, n1, n2))
                                         append(q, rank);
                             });
            }
        }, [] {});
    }
    __syncthreads();
    const int sx = 2 * int(b % nbx) + (w & 1), sy = 2 * int(b / nbx) + (w >> 1);
    if (sx < nsx && sy < nsy) {
        const int64_t sidx = int64_t(sy) * nsx + sx;
        const uint32_t cnt = sh.qn[w];
        const bool keep = cnt <= uint32_t(A.depth);
        char* bb = reinterpret_cast<char*>(A.bins);
        uint32_t* out = reinterpret_cast<uint32_t*>(bb + 256 + align256(A.ntiles * 4)) + sidx * A.depth;
        if (keep) bucket_sort_wave(qlist + w * lcap, cnt, sh.g.bk[w], bucket_shift(A.n), out);
        if (lane == 0) {
            reinterpret_cast<uint32_t*>(bb + 256)[sidx] = cnt;
            if (!keep) atomicAdd(A.status, 1u);
        }
    }
}

// The 16x16-tile block binners are held to 64 VGPRs, so that a SIMD runs 8
// of their waves (its maximum) instead of the 7 that their 71 registers
// allow: one register and a few scalars spill, and the binner's time on 64
// views of 1920x1080 drops by 5% (its chain of loads and barriers per
// workgroup overlaps with more workgroups).
#define VSR_BLOCK16_WAVES __attribute__((amdgpu_waves_per_eu(8, 8)))

__global__ __launch_bounds__(256) VSR_BLOCK16_WAVES void k_bin_block16(BinArgs A) {
    bin_block16(A, xcd_remap(blockIdx.x, gridDim.x));
}

// Automatic binner shape: 32x32 blocks for list capacities up to
// kBlockMaxCap and launches of at least kBlockMinGrid blocks.  Below that a
// block's longer candidate stream leaves the chip under-filled (the slowest
// blocks set the launch time): on the 1M-triangle scene the shapes tie at
// 1600x900 and 1920x1080 (1,450 and 2,040 blocks; at 1920x1080 blocks are
// 0.90x over four perspective lenses but a 2048x1024 equirectangular map,
// whose polar blocks gather far more, takes 1.35x), blocks take 0.81x the
// super-tiles' time at 2560x1440 and 0.67x at 3840x2160.
constexpr int32_t kBlockMaxCap = 256;
constexpr int32_t kBlock16MaxCap = 1024;  // four LDS lists of this many entries
constexpr int64_t kBlockMinGrid = 2560;

inline bool use_blocks(int32_t lds_cap, int64_t nblk, uint32_t flags, bool tile16 = false) {
    // 8x8 lists: blocks sort lists of at most 256 in registers
    if (lds_cap > (tile16 ? kBlock16MaxCap : kBlockMaxCap)) return false;
    if (flags & VSR_BIN_BLOCKS) return true;
    if (flags & VSR_BIN_SUPERTILES) return false;
    return nblk >= kBlockMinGrid;
}

__global__ __launch_bounds__(64) void k_zero_u32(uint32_t* p, int64_t n) {
    int64_t i = int64_t(blockIdx.x) * 64 + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// Status header of a bin buffer: word 0 counts overflowed lists, word 1
// records the bin tile edge (8 or 16) for the rasterizer.
constexpr int kBinHdrTile = 1;
__global__ __launch_bounds__(64) void k_bins_header(uint32_t* hdr, uint32_t tile) {
    hdr[threadIdx.x] = threadIdx.x == kBinHdrTile ? tile : 0u;
}

inline int32_t bin_lds_cap(int32_t depth) {
    int32_t c = 64;
    while (c < depth) c <<= 1;
    return c;
}

inline int64_t bin_grid(int32_t ntx, int32_t nty) { return int64_t((ntx + 1) / 2) * ((nty + 1) / 2); }

hipError_t launch_bin(const void* map, int32_t W, int32_t H, int32_t fmt, const Rot& R, const void* setup, int64_t n,
                      int32_t depth, uint32_t flags, void* bins, hipStream_t st) {
    MapLayout ML = map_layout(W, H, fmt);
    BinArgs A;
    A.map = map;
    A.ntiles = ML.ntiles;
    A.fmt = fmt;
    A.depth = depth;
    A.lds_cap = bin_lds_cap(depth);
    A.all = (flags & VSR_BIN_ALL) ? 1 : 0;
    A.ntx = ML.ntx;
    A.nty = ML.nty;
    A.setup = setup;
    A.n = n;
    A.bins = bins;
    A.status = reinterpret_cast<uint32_t*>(bins);
    A.rot = R;
    A.tile16 = (flags & VSR_BIN_TILE16) ? 1 : 0;
    A.pad = 0;
    hipLaunchKernelGGL(k_bins_header, dim3(1), dim3(64), 0, st, reinterpret_cast<uint32_t*>(bins),
                       uint32_t(A.tile16 ? 16 : 8));
    if (A.tile16) {
        if (use_blocks(A.lds_cap, ML.nblk, flags, true))
            hipLaunchKernelGGL(k_bin_block16, dim3(unsigned(ML.nblk)), dim3(256), size_t(4) * A.lds_cap * 4, st, A);
        else
            hipLaunchKernelGGL(k_bin16, dim3(unsigned(bin_grid(ML.ntx, ML.nty))), dim3(256), size_t(A.lds_cap) * 4,
                               st, A);
    } else if (use_blocks(A.lds_cap, ML.nblk, flags)) {
        hipLaunchKernelGGL(k_bin_block, dim3(unsigned(ML.nblk)), dim3(256), 0, st, A);
    } else {
        hipLaunchKernelGGL(k_bin, dim3(unsigned(bin_grid(ML.ntx, ML.nty))), dim3(256),
                           size_t(kSupTiles) * A.lds_cap * 4, st, A);
    }
    return hipGetLastError();
}

}  // namespace vsr
