// Per-pixel edge-plane rasterization with depth test.
//
// One 64-lane wavefront per 8x8 tile; each lane owns one pixel direction g
// and a 64-bit z-buffer key (depth bits << 32 | triangle id).  For every
// listed triangle the lane forms the three oriented edge-plane values
// n_i . g (section 1.1); all three > 0 is the binary step of section 1.1.1.
// Covered lanes take r = d / (g . N) (section 1.1.4) and keep the smaller key
// (depth-pass test, section 1.4; ties to the lower id).
//
// Records are fetched 16 at a time: lane l loads float4 (l & 3) of triangle
// (l >> 2) of the group, one vector load for the whole wave, staged in LDS
// and read back as wave-wide broadcasts; the next group is in flight while
// one is tested.  Lists are in depth-bucket order (nearest first): once
// every pixel of the tile holds a depth below the lower bound of the
// current bucket, no later triangle can win and the wave stops.  With 16x16
// bin tiles a wave takes a 16x8 strip, two pixels per lane (see below).
#pragma once
#include "bin.hpp"

namespace vsr {

// ------------------------------------------------------------- raster ---
struct RasterArgs {
    const void* map;
    int64_t ntiles;
    int32_t fmt, depth, W, H, ntx, nty;
    const void* setup;
    int64_t n;
    const void* bins;
    uint32_t* tri_id;
    float* out_depth;
    unsigned long long* stats;  // instrumented variant only: tests, covered, triangles, tiles
    int32_t no_early_exit;      // instrumented variant only: process whole lists
    Rot rot;                    // camera -> world

    __device__ inline void globalize() {
        map = to_global(map);
        setup = to_global(setup);
        bins = to_global(bins);
        tri_id = to_global(tri_id);
        out_depth = to_global(out_depth);
        stats = to_global(stats);
    }
};

// One triangle (record r0..r3) against the lane's pixel; returns whether it
// covers it.
__device__ inline bool raster_rec(float4 r0, float4 r1, float4 r2, float4 r3, float3 g, uint64_t& best) {
    float e0 = fmaf(r0.z, g.z, fmaf(r0.y, g.y, r0.x * g.x));
    float e1 = fmaf(r1.z, g.z, fmaf(r1.y, g.y, r1.x * g.x));
    float e2 = fmaf(r2.z, g.z, fmaf(r2.y, g.y, r2.x * g.x));
    if (fminf(e0, fminf(e1, e2)) > 0.0f) {
        float dn = fmaf(r2.w, g.z, fmaf(r1.w, g.y, r0.w * g.x));
        if (dn > 0.0f) {
            float rr = r3.x * __builtin_amdgcn_rcpf(dn);
            uint64_t key = (uint64_t(__float_as_uint(rr)) << 32) | uint64_t(__float_as_uint(r3.z));
            best = key < best ? key : best;
            return true;
        }
    }
    return false;
}

__device__ inline bool raster_one(const float4* __restrict__ rec, uint32_t rank, float3 g, uint64_t& best) {
    const float4* r = rec + 4 * int64_t(rank);
    return raster_rec(r[0], r[1], r[2], r[3], g, best);
}

// Tests the `count` triangles whose ranks are lst[0..count) against the
// lane's pixel (all lanes of the wave call it with the same list).  With
// early_exit, stops once every pixel with a direction holds a depth below
// the current triangle's bucket bound.  Returns true when it stopped early.
// pre0/pre1 are lst[sub] and lst[16 + sub] (sub = lane / 4) when the
// caller loaded them already (each only read where below count).
template <bool kStats>
__device__ inline bool raster_list(const uint32_t* lst, uint32_t count, const float4* __restrict__ rec, float3 g,
                                   bool has_dir, uint64_t& best, float4* stg, bool early_exit,
                                   unsigned long long& n_tri, unsigned long long& n_cov, const uint32_t* pre = nullptr) {
    const int lane = threadIdx.x & 63;
    const uint32_t ngroups = (count + 15u) >> 4;
    const uint32_t sub = uint32_t(lane) >> 2, part = uint32_t(lane) & 3u;
    uint32_t rk = sub < count ? (pre ? pre[0] : lst[sub]) : 0u;
    float4 v = rec[4 * int64_t(rk) + part];
    rk = 16u + sub < count ? (pre ? pre[1] : lst[16u + sub]) : 0u;
    bool done = false;
    for (uint32_t gi = 0; gi < ngroups && !done; ++gi) {
        stg[lane] = v;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (gi + 1 < ngroups) v = rec[4 * int64_t(rk) + part];
        if (gi + 2 < ngroups) {
            uint32_t e = (gi + 2) * 16u + sub;
            rk = e < count ? lst[e] : 0u;
        }
        const uint32_t nt = min(16u, count - gi * 16u);
        // the early exit is checked every 4 triangles (1080p x 1M: 6% faster
        // than every 8; every 2 gains nothing more, every 16 loses 15%)
        for (uint32_t t8 = 0; t8 < nt; t8 += 4) {
            if (early_exit) {
                // every pixel already beats the depth lower bound of this
                // triangle's bucket, which bounds every triangle still to come
                // (the builtin takes an int: pass the bits, not the value)
                const float lb = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(stg[4 * t8 + 3].w)));
                const bool below = !has_dir || __uint_as_float(uint32_t(best >> 32)) < lb;
                if (__ballot(!below) == 0) {
                    done = true;
                    break;
                }
            }
#pragma unroll
            for (uint32_t u = 0; u < 4; ++u) {
                const uint32_t t = t8 + u;
                if (t < nt) {
                    float4 c0 = stg[4 * t], c1 = stg[4 * t + 1], c2 = stg[4 * t + 2], c3 = stg[4 * t + 3];
                    bool cov = raster_rec(c0, c1, c2, c3, g, best);
                    if (kStats) {
                        n_tri += 1;
                        n_cov += __popcll(__ballot(cov));
                    }
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
    return done;
}

template <bool kStats>
__device__ inline void raster_tile(const RasterArgs& A0, int64_t tile, int lane) {
    RasterArgs A = A0;
    A.globalize();
    const float4* caps = map_caps(A.map, A.ntiles, A.fmt);
    SceneView S = scene_view(A.setup, A.n);
    const char* bb = reinterpret_cast<const char*>(A.bins);
    const uint32_t* counts = reinterpret_cast<const uint32_t*>(bb + 256);
    const uint32_t* lists = reinterpret_cast<const uint32_t*>(bb + 256 + align256(A.ntiles * 4));

    int tx = int(tile % A.ntx), ty = int(tile / A.ntx);
    int i = tx * kTile + (lane & (kTile - 1)), j = ty * kTile + (lane >> 3);
    bool inside = i < A.W && j < A.H;
    float3 g = load_dir(A.map, A.fmt, A.ntiles, tile, lane, A.rot);
    bool has_dir = inside && (g.x != 0.0f || g.y != 0.0f || g.z != 0.0f);
    uint64_t best = kKeyEmpty;
    // the first list words are requested together with the count (in
    // bounds whatever the count; used only below it), one round trip less
    const uint32_t* lst = lists + tile * A.depth;
    const uint32_t dm = uint32_t(A.depth) - 1u, sub = uint32_t(lane) >> 2;
    const uint32_t pre[2] = {lst[min(sub, dm)], lst[min(16u + sub, dm)]};
    const uint32_t count = __builtin_amdgcn_readfirstlane(counts[tile]);  // uniform: scalar loop bounds
    asm volatile("" ::"v"(pre[0]), "v"(pre[1]), "s"(count));  // in flight together
    unsigned long long n_tri = 0, n_cov = 0;
    if (count <= uint32_t(A.depth)) {
        __shared__ float4 s_stage[4][64];
        raster_list<kStats>(lst, count, S.rec, g, has_dir, best, s_stage[threadIdx.x >> 6],
                            !(kStats && A.no_early_exit), n_tri, n_cov, pre);
    } else {
        float4 tc0, tc1;
        load_tile_cap(caps, tile, A.rot, tc0, tc1);
        gather_candidates(S, tc0, tc1, lane, [&](uint32_t rank, bool valid) {
            bool pass = valid && candidate_test(S, rank, tc0, tc1);
            uint64_t m = __ballot(pass);
            while (m) {
                int q = __ffsll((unsigned long long)m) - 1;
                m &= m - 1;
                uint32_t rk = uint32_t(__builtin_amdgcn_readlane(int(rank), q));
                bool cov = raster_one(S.rec, rk, g, best);
                if (kStats) {
                    n_tri += 1;
                    n_cov += __popcll(__ballot(cov));
                }
            }
        });
    }
    unsigned long long npix = kStats ? (unsigned long long)__popcll(__ballot(has_dir)) : 0ull;
    if (kStats && lane == 0) {
        atomicAdd(&A.stats[0], n_tri * npix);
        atomicAdd(&A.stats[1], n_cov);
        atomicAdd(&A.stats[2], n_tri);
        atomicAdd(&A.stats[3], 1ull);
    }
    if (inside) {
        int64_t o = int64_t(j) * A.W + i;
        A.tri_id[o] = uint32_t(best & 0xFFFFFFFFull);
        A.out_depth[o] = __uint_as_float(uint32_t(best >> 32));
    }
}

// ------------------------------------------------ 16x16 bin tiles ------
// One wave per 8x8 tile of a super-tile (the persistent rasterizer's work
// item; the grid kernels use the two-pixel strips below).  The wave walks
// the super-tile's list in chunks of 64: lane l takes entry l, with its
// binning cap (rank order) and record, and keeps it when sub_may_see passes
// for the tile's cap — the test the 8x8 binner applies, on the same cap and
// normals, so the survivors are that binner's list for the tile, in the same
// depth-bucket order.  Survivors' records are compacted into LDS (word k of
// survivor p at stg[64 k + p]) and tested as in raster_list (same early
// exit).  A chunk is loaded only when the previous one did not end the tile:
// most tiles stop within the first 64 entries, so loading the next chunk
// ahead would mostly fetch entries nobody tests (measured: 32% slower).
template <bool kStats>
__device__ inline void raster_list_cull(const uint32_t* lst, uint32_t count, const SceneView& S, float4 tc0,
                                        float4 tc1, float3 g, bool has_dir, uint64_t& best, float4* stg,
                                        bool early_exit, unsigned long long& n_tri, unsigned long long& n_cov,
                                        uint32_t pre) {
    // pre: lst[lane], loaded by the caller with the count (read below it only)
    const int lane = threadIdx.x & 63;
    for (uint32_t c0 = 0; c0 < count; c0 += 64) {
        if (c0 > 0 && early_exit) {
            // before loading a chunk: every pixel may already beat the bucket
            // bound of its first entry, which bounds all that follow
            const uint32_t r0k = __builtin_amdgcn_readfirstlane(lst[c0]);
            const float lb0 = S.rec[4 * int64_t(r0k) + 3].w;
            if (__ballot(has_dir && !(__uint_as_float(uint32_t(best >> 32)) < lb0)) == 0) break;
        }
        const bool valid = c0 + uint32_t(lane) < count;
        const uint32_t rank = c0 == 0 ? (valid ? pre : 0u) : lst[min(c0 + uint32_t(lane), count - 1u)];
        const float4 a = S.rcap[rank];
        const float4* rp = S.rec + 4 * int64_t(rank);
        const float4 r0 = rp[0], r1 = rp[1], r2 = rp[2], r3 = rp[3];
        const bool pass = valid && sub_may_see_lazy(tc0, tc1, a, bin_cos_half(a), f3(r0.x, r0.y, r0.z),
                                               f3(r1.x, r1.y, r1.z), f3(r2.x, r2.y, r2.z));
        const uint64_t bal = __ballot(pass);
        const uint32_t ns = uint32_t(__popcll(bal));
        if (pass) {
            // word k of survivor p at stg[64 k + p]: consecutive lanes write
            // consecutive 16-byte slots (no bank conflicts)
            const uint32_t pos =
                __builtin_amdgcn_mbcnt_hi(uint32_t(bal >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(bal), 0u));
            stg[pos] = r0;
            stg[64 + pos] = r1;
            stg[128 + pos] = r2;
            stg[192 + pos] = r3;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        bool done = false;
        for (uint32_t t8 = 0; t8 < ns; t8 += 4) {
            if (early_exit) {
                const float lb = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(stg[192 + t8].w)));
                const bool below = !has_dir || __uint_as_float(uint32_t(best >> 32)) < lb;
                if (__ballot(!below) == 0) {
                    done = true;
                    break;
                }
            }
#pragma unroll
            for (uint32_t u = 0; u < 4; ++u) {
                const uint32_t t = t8 + u;
                if (t < ns) {
                    float4 c0v = stg[t], c1v = stg[64 + t], c2v = stg[128 + t], c3v = stg[192 + t];
                    bool cov = raster_rec(c0v, c1v, c2v, c3v, g, best);
                    if (kStats) {
                        n_tri += 1;
                        n_cov += __popcll(__ballot(cov));
                    }
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        if (done) break;
    }
}

template <bool kStats>
__device__ inline void raster_quad16(const RasterArgs& A0, int64_t sidx, int w, float4* stg) {
    RasterArgs A = A0;
    A.globalize();
    const int lane = threadIdx.x & 63;
    int64_t tile;
    int tx, ty;
    if (!super_tile_of(sidx, w, A.ntx, A.nty, tile, tx, ty)) return;
    const float4* caps = map_caps(A.map, A.ntiles, A.fmt);
    SceneView S = scene_view(A.setup, A.n);
    const char* bb = reinterpret_cast<const char*>(A.bins);
    const uint32_t* counts = reinterpret_cast<const uint32_t*>(bb + 256);
    const uint32_t* lists = reinterpret_cast<const uint32_t*>(bb + 256 + align256(A.ntiles * 4));
    const int i = tx * kTile + (lane & (kTile - 1)), j = ty * kTile + (lane >> 3);
    const bool inside = i < A.W && j < A.H;
    const float3 g = load_dir(A.map, A.fmt, A.ntiles, tile, lane, A.rot);
    const bool has_dir = inside && (g.x != 0.0f || g.y != 0.0f || g.z != 0.0f);
    float4 tc0, tc1;
    load_tile_cap(caps, tile, A.rot, tc0, tc1);
    uint64_t best = kKeyEmpty;
    unsigned long long n_tri = 0, n_cov = 0;
    // the first 64 list words are requested together with the count (in
    // bounds whatever the count; used only below it), one round trip less
    const uint32_t* lst = lists + sidx * A.depth;
    const uint32_t pre = lst[min(uint32_t(lane), uint32_t(A.depth) - 1u)];
    const uint32_t count = __builtin_amdgcn_readfirstlane(counts[sidx]);
    // both in flight together (the compiler would sink the list load into
    // the branch that uses it, after the count has arrived)
    asm volatile("" ::"v"(pre), "s"(count));
    if (count <= uint32_t(A.depth)) {
        if (count > 0 && tc1.z != kCapEmpty)
            raster_list_cull<kStats>(lst, count, S, tc0, tc1, g, has_dir, best, stg, !(kStats && A.no_early_exit),
                                     n_tri, n_cov, pre);
    } else {
        // overflowed list: the tile gathers its own candidates
        gather_candidates(S, tc0, tc1, lane, [&](uint32_t rank, bool valid) {
            bool pass = valid && candidate_test(S, rank, tc0, tc1);
            uint64_t mm = __ballot(pass);
            while (mm) {
                int q = __ffsll((unsigned long long)mm) - 1;
                mm &= mm - 1;
                uint32_t rk = uint32_t(__builtin_amdgcn_readlane(int(rank), q));
                bool cov = raster_one(S.rec, rk, g, best);
                if (kStats) {
                    n_tri += 1;
                    n_cov += __popcll(__ballot(cov));
                }
            }
        });
    }
    const unsigned long long npix = kStats ? (unsigned long long)__popcll(__ballot(has_dir)) : 0ull;
    if (kStats && lane == 0) {
        atomicAdd(&A.stats[0], n_tri * npix);
        atomicAdd(&A.stats[1], n_cov);
        atomicAdd(&A.stats[2], n_tri);
        atomicAdd(&A.stats[3], 1ull);
    }
    if (inside) {
        int64_t o = int64_t(j) * A.W + i;
        A.tri_id[o] = uint32_t(best & 0xFFFFFFFFull);
        A.out_depth[o] = __uint_as_float(uint32_t(best >> 32));
    }
}

// Grid kernels: a super-tile's 16x16 pixels are two 16x8 strips, one wave
// each; a lane owns pixel (l & 7, l >> 3) of both 8x8 tiles of its strip (A
// on the left, B on the right), so every record broadcast from LDS serves
// two pixel tests, and the list, map and cap loads and the cull serve twice
// the pixels.  A triangle kept for one tile of the strip is also tested on
// the other (exactly, finding nothing there), and the strip ends when both
// tiles' pixels are done: 35 triangles per strip against 2 x 12.6 per tile
// on the benchmark views, yet faster than a wave per tile (1.75 against
// 2.09 ms per 64 views).  The per-pixel flags combine bitwise, without
// short-circuit branches (9% of that gain).  The cull keeps an entry when
// sub_may_see_lazy passes for either tile's cap, so the
// survivors are the union of the 8x8 binner's two lists, in the same
// depth-bucket order; they are compacted into LDS as above and tested with
// the early exit taken when both pixels of every lane beat the bound.

// Pixels of a lane when a wave covers NP 8x8 tiles: pixel p lies in tile p.
template <int NP>
struct LanePix {
    float3 g[NP];
    bool dir[NP];
    uint64_t best[NP];
};

// One triangle (record r0..r3) against the lane's NP pixels; the arithmetic
// for each pixel is raster_rec's, so the images are the same bit for bit.
// Returns the mask of the pixels it covers (for the statistics).
// Only the tiles whose bit is set in the wave-uniform mask `live` are
// tested: the others are done (every pixel already beats the depth bound of
// the current group, which bounds this triangle).
template <int NP>
__device__ inline uint32_t raster_rec_n(float4 r0, float4 r1, float4 r2, float4 r3, LanePix<NP>& P, uint32_t live) {
    // smallest edge value per pixel (-1: not tested), kept as values rather
    // than flags so that a skipped tile costs one move
    float em[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        em[p] = -1.0f;
        if (live & (1u << p)) {
            const float3 g = P.g[p];
            const float e0 = fmaf(r0.z, g.z, fmaf(r0.y, g.y, r0.x * g.x));
            const float e1 = fmaf(r1.z, g.z, fmaf(r1.y, g.y, r1.x * g.x));
            const float e2 = fmaf(r2.z, g.z, fmaf(r2.y, g.y, r2.x * g.x));
            em[p] = fminf(e0, fminf(e1, e2));
        }
    }
    bool any = false;
#pragma unroll
    for (int p = 0; p < NP; ++p) any |= em[p] > 0.0f;
    uint32_t cov = 0;
    if (any) {
        const uint64_t idk = uint64_t(__float_as_uint(r3.z));
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            const float3 g = P.g[p];
            const float dn = fmaf(r2.w, g.z, fmaf(r1.w, g.y, r0.w * g.x));
            if ((em[p] > 0.0f) & (dn > 0.0f)) {
                const float rr = r3.x * __builtin_amdgcn_rcpf(dn);
                const uint64_t key = (uint64_t(__float_as_uint(rr)) << 32) | idk;
                P.best[p] = key < P.best[p] ? key : P.best[p];
                cov |= 1u << p;
            }
        }
    }
    return cov;
}

// Can a later triangle with depth lower bound lb still win a pixel of the
// lane?  (Pixels without a direction never wait.)
template <int NP>
__device__ inline bool lane_open(const LanePix<NP>& P, float lb) {
    bool open = false;
#pragma unroll
    for (int p = 0; p < NP; ++p) open |= P.dir[p] && !(__uint_as_float(uint32_t(P.best[p] >> 32)) < lb);
    return open;
}

template <bool kStats, int NP>
__device__ inline void raster_list_cull_n(const uint32_t* lst, uint32_t count, const SceneView& S,
                                          const float4 (&tc0)[NP], const float4 (&tc1)[NP], LanePix<NP>& P,
                                          float4* stg, bool early_exit, unsigned long long& n_tri,
                                          unsigned long long& n_cov, uint32_t pre) {
    // pre: lst[lane], loaded by the caller with the count (read below it only)
    const int lane = threadIdx.x & 63;
    for (uint32_t c0 = 0; c0 < count; c0 += 64) {
        if (c0 > 0 && early_exit) {
            // before loading a chunk: every pixel may already beat the bucket
            // bound of its first entry, which bounds all that follow
            const uint32_t r0k = __builtin_amdgcn_readfirstlane(lst[c0]);
            const float lb0 = S.rec[4 * int64_t(r0k) + 3].w;
            if (__ballot(lane_open(P, lb0)) == 0) break;
        }
        const bool valid = c0 + uint32_t(lane) < count;
        const uint32_t rank = c0 == 0 ? (valid ? pre : 0u) : lst[min(c0 + uint32_t(lane), count - 1u)];
        const float4 a = S.rcap[rank];
        const float4* rp = S.rec + 4 * int64_t(rank);
        const float4 r0 = rp[0], r1 = rp[1], r2 = rp[2], r3 = rp[3];
        const float ch = bin_cos_half(a);
        const float3 n0 = f3(r0.x, r0.y, r0.z), n1 = f3(r1.x, r1.y, r1.z), n2 = f3(r2.x, r2.y, r2.z);
        bool pass = false;
#pragma unroll
        for (int p = 0; p < NP; ++p) pass |= sub_may_see_lazy(tc0[p], tc1[p], a, ch, n0, n1, n2);
        pass = pass && valid;
        const uint64_t bal = __ballot(pass);
        const uint32_t ns = uint32_t(__popcll(bal));
        if (pass) {
            const uint32_t pos =
                __builtin_amdgcn_mbcnt_hi(uint32_t(bal >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(bal), 0u));
            stg[pos] = r0;
            stg[64 + pos] = r1;
            stg[128 + pos] = r2;
            stg[192 + pos] = r3;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        bool done = false;
        for (uint32_t t8 = 0; t8 < ns; t8 += 4) {
            // tiles whose pixels may still change (all without the exit)
            uint32_t live = (1u << NP) - 1u;
            if (early_exit) {
                const float lb = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(stg[192 + t8].w)));
                live = 0;
#pragma unroll
                for (int p = 0; p < NP; ++p)
                    live |= __ballot(P.dir[p] && !(__uint_as_float(uint32_t(P.best[p] >> 32)) < lb)) ? 1u << p : 0u;
                if (live == 0) {
                    done = true;
                    break;
                }
            }
#pragma unroll
            for (uint32_t u = 0; u < 4; ++u) {
                const uint32_t t = t8 + u;
                if (t < ns) {
                    const uint32_t cov =
                        raster_rec_n<NP>(stg[t], stg[64 + t], stg[128 + t], stg[192 + t], P, live);
                    if (kStats) {
                        n_tri += 1;
#pragma unroll
                        for (int p = 0; p < NP; ++p) n_cov += __popcll(__ballot((cov >> p) & 1u));
                    }
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        if (done) break;
    }
}

// Overflowed list: the tile (cap tc0/tc1, lane pixel g) gathers its own
// candidates from the cap index.
template <bool kStats>
__device__ inline void raster_gather_tile(const SceneView& S, float4 tc0, float4 tc1, float3 g, int lane,
                                          uint64_t& best, unsigned long long& n_tri, unsigned long long& n_cov) {
    gather_candidates(S, tc0, tc1, lane, [&](uint32_t rank, bool valid) {
        bool pass = valid && candidate_test(S, rank, tc0, tc1);
        uint64_t mm = __ballot(pass);
        while (mm) {
            int q = __ffsll((unsigned long long)mm) - 1;
            mm &= mm - 1;
            uint32_t rk = uint32_t(__builtin_amdgcn_readlane(int(rank), q));
            bool cov = raster_one(S.rec, rk, g, best);
            if (kStats) {
                n_tri += 1;
                n_cov += __popcll(__ballot(cov));
            }
        }
    });
}

// Grid kernels with 16x16 lists: each wave takes kStripTiles 8x8 tiles of a
// super-tile (its `part`-th row for 2, all four for 4); stg is the wave's
// 4 KB of LDS.
constexpr int kStripTiles = 2;

template <bool kStats, int NP>
__device__ inline void raster_multi16(const RasterArgs& A0, int64_t sidx, int part, float4* stg) {
    RasterArgs A = A0;
    A.globalize();
    const int lane = threadIdx.x & 63;
    const float4* caps = map_caps(A.map, A.ntiles, A.fmt);
    SceneView S = scene_view(A.setup, A.n);
    const char* bb = reinterpret_cast<const char*>(A.bins);
    const uint32_t* counts = reinterpret_cast<const uint32_t*>(bb + 256);
    const uint32_t* lists = reinterpret_cast<const uint32_t*>(bb + 256 + align256(A.ntiles * 4));
    LanePix<NP> P;
    float4 tc0[NP], tc1[NP];
    int64_t tile[NP];
    int px[NP], py[NP];
    bool inside[NP], has[NP], any_tile = false;
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        int tx, ty;
        const int q = NP == 4 ? p : 2 * part + p;  // quadrant of the super-tile
        has[p] = super_tile_of(sidx, q, A.ntx, A.nty, tile[p], tx, ty);
        px[p] = tx * kTile + (lane & (kTile - 1));
        py[p] = ty * kTile + (lane >> 3);
        inside[p] = has[p] && px[p] < A.W && py[p] < A.H;
        P.g[p] = has[p] ? load_dir(A.map, A.fmt, A.ntiles, tile[p], lane, A.rot) : f3(0.0f, 0.0f, 0.0f);
        P.dir[p] = inside[p] && (P.g[p].x != 0.0f || P.g[p].y != 0.0f || P.g[p].z != 0.0f);
        P.best[p] = kKeyEmpty;
        tc0[p] = empty_cap0();
        tc1[p] = empty_cap1();
        if (has[p]) load_tile_cap(caps, tile[p], A.rot, tc0[p], tc1[p]);
        any_tile |= has[p];
    }
    if (!any_tile) return;
    unsigned long long n_tri = 0, n_cov = 0;
    const uint32_t* lst = lists + sidx * A.depth;
    const uint32_t pre = lst[min(uint32_t(lane), uint32_t(A.depth) - 1u)];
    const uint32_t count = __builtin_amdgcn_readfirstlane(counts[sidx]);
    asm volatile("" ::"v"(pre), "s"(count));  // in flight together
    unsigned long long npix = 0;
    if (kStats) {
#pragma unroll
        for (int p = 0; p < NP; ++p) npix += __popcll(__ballot(P.dir[p]));
    }
    if (count <= uint32_t(A.depth)) {
        bool live = false;
#pragma unroll
        for (int p = 0; p < NP; ++p) live |= tc1[p].z != kCapEmpty;
        if (count > 0 && live)
            raster_list_cull_n<kStats, NP>(lst, count, S, tc0, tc1, P, stg, !(kStats && A.no_early_exit), n_tri,
                                           n_cov, pre);
        if (kStats && lane == 0) atomicAdd(&A.stats[0], n_tri * npix);
    } else {
        // each tile gathers and counts its own candidates
#pragma unroll
        for (int p = 0; p < NP; ++p) {
            unsigned long long nt = 0;
            raster_gather_tile<kStats>(S, tc0[p], tc1[p], P.g[p], lane, P.best[p], nt, n_cov);
            if (kStats) {
                const unsigned long long pp = __popcll(__ballot(P.dir[p]));
                if (lane == 0) atomicAdd(&A.stats[0], nt * pp);
                n_tri += nt;
            }
        }
    }
    if (kStats && lane == 0) {
        unsigned long long ntiles = 0;
#pragma unroll
        for (int p = 0; p < NP; ++p) ntiles += has[p] ? 1ull : 0ull;
        atomicAdd(&A.stats[1], n_cov);
        atomicAdd(&A.stats[2], n_tri);
        atomicAdd(&A.stats[3], ntiles);
    }
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        if (inside[p]) {
            const int64_t o = int64_t(py[p]) * A.W + px[p];
            A.tri_id[o] = uint32_t(P.best[p] & 0xFFFFFFFFull);
            A.out_depth[o] = __uint_as_float(uint32_t(P.best[p] >> 32));
        }
    }
}

// Plain rasterizer: the bin buffer's header says whether its lists are per
// 8x8 tile (workgroups of 4 consecutive tiles) or per 16x16 super-tile (one
// workgroup per super-tile); the grid covers the larger of the two counts.
template <bool kStats>
__global__ __launch_bounds__(256) void k_raster(RasterArgs A) {
    const bool b16 = reinterpret_cast<const uint32_t*>(A.bins)[kBinHdrTile] == 16u;
    if (b16) {
        // kStripTiles super-tiles per workgroup, 4 / kStripTiles waves each
        constexpr int kWps = 4 / kStripTiles;
        __shared__ float4 s_stage16[4][256];
        const int w = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
        const int64_t nsx = (A.ntx + 1) / 2, nsup = nsx * ((A.nty + 1) / 2);
        const int64_t s = kStripTiles * int64_t(blockIdx.x) + w / kWps;
        if (s >= nsup) return;
        raster_multi16<kStats, kStripTiles>(A, band_remap(s, nsup, max(int64_t(1), nsx * kBandPx / (2 * kTile))),
                                            w % kWps, s_stage16[w]);
        return;
    }
    const int64_t nwg = (A.ntiles + 3) / 4;
    if (int64_t(blockIdx.x) >= nwg) return;
    int w = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    // workgroups of 4 consecutive tiles, ntx tiles per row
    int64_t tile = band_remap(blockIdx.x, nwg, max(int64_t(1), int64_t(A.ntx) * kBandPx / (4 * kTile))) * 4 + w;
    if (tile >= A.ntiles) return;
    raster_tile<kStats>(A, tile, threadIdx.x & 63);
}

hipError_t launch_raster(const void* map, int32_t W, int32_t H, int32_t fmt, const Rot& R, const void* setup, int64_t n,
                         const void* bins, int32_t depth, uint32_t* tri_id, float* out_depth, hipStream_t st,
                         unsigned long long* stats = nullptr, int32_t no_early_exit = 0) {
    MapLayout ML = map_layout(W, H, fmt);
    RasterArgs A;
    A.map = map;
    A.ntiles = ML.ntiles;
    A.fmt = fmt;
    A.depth = depth;
    A.W = W;
    A.H = H;
    A.ntx = ML.ntx;
    A.nty = ML.nty;
    A.setup = setup;
    A.n = n;
    A.bins = bins;
    A.tri_id = tri_id;
    A.out_depth = out_depth;
    A.stats = stats;
    A.no_early_exit = no_early_exit;
    A.rot = R;
    // 4 tiles per workgroup (8x8 lists) or kStripTiles super-tiles (16x16 lists)
    const int64_t nsup = int64_t((ML.ntx + 1) / 2) * ((ML.nty + 1) / 2);
    int64_t blocks = std::max((ML.ntiles + 3) / 4, (nsup + kStripTiles - 1) / kStripTiles);
    if (stats) {
        hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, reinterpret_cast<uint32_t*>(stats), int64_t(8));
        hipLaunchKernelGGL(k_raster<true>, dim3(unsigned(blocks)), dim3(256), 0, st, A);
    } else {
        hipLaunchKernelGGL(k_raster<false>, dim3(unsigned(blocks)), dim3(256), 0, st, A);
    }
    return hipGetLastError();
}

}  // namespace vsr
