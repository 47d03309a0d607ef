// Conservative binning and the per-pixel edge-plane rasterizer.
//
// Both kernels give one 64-lane wavefront to one 8x8 tile.
//
// Gathering (shared by the binner and by the rasterizer's overflow path):
// a tile's cap (centre c, radius rho) can only meet the cap of a triangle
// filed at index level L (cap radius <= R_L) if the triangle's cap centre
// lies within rho + R_L of c.  Lane p of the wave computes, for level p/6 and
// cube face p%6, the rectangle of cells that such centres can occupy (from
// the longitude/latitude extent of a spherical cap); every row of that
// rectangle is one contiguous run of the cell-sorted triangle list.  Runs are
// streamed 64 candidates at a time, one per lane, through the conservative
// cap and edge-plane test; survivors are compacted with ballot + mbcnt.
//
// Binning keeps the survivors in LDS and writes each tile's list ordered by
// depth bucket (triangle ranks are nearest-first; a bucket is a run of
// consecutive ranks) with a counting sort.
//
// Rasterization: each lane owns one pixel direction g and a 64-bit z-buffer
// key (depth bits << 32 | triangle id).  For every listed triangle, staged
// through LDS and read as wave-wide broadcasts, the lane forms the three
// oriented edge-plane values n_i . g (section 1.1); all three > 0 is the
// binary step of section 1.1.1.  Covered lanes take r = d / (g . N)
// (section 1.1.4) and keep the smaller key (depth-pass test, section 1.4;
// ties to the lower id).  Lists are in bucket order: once every pixel of the
// tile holds a depth below the lower bound of the current bucket, no later
// triangle can win and the wave stops.
#pragma once
#include "vsr_internal.h"

namespace vsr {

struct SceneView {
    const float4* rec;         // 4 x float4 per triangle, nearest-first order
    const float4* cap;         // 2 x float4 per triangle
    const uint32_t* cell_list; // ranks sorted by cell
    const uint32_t* cell_start;
    int64_t n;
};

__device__ inline SceneView scene_view(const void* setup, int64_t n) {
    SetupLayout L = setup_layout(n);
    const char* b = reinterpret_cast<const char*>(setup);
    SceneView s;
    s.rec = reinterpret_cast<const float4*>(b + L.rec_off);
    s.cap = reinterpret_cast<const float4*>(b + L.cap_off);
    s.cell_list = reinterpret_cast<const uint32_t*>(b + L.cell_list_off);
    s.cell_start = reinterpret_cast<const uint32_t*>(b + L.cell_start_off);
    s.n = n;
    return s;
}

// Longitude range of a cap (centre with components p along the measured
// axis, q along the face normal, r along the rotation axis; radius alpha),
// intersected with the face's [-pi/4, pi/4].  False when empty.
__device__ inline bool lon_range(float p, float q, float r, float alpha, float& lo, float& hi) {
    float lam = atan2f(p, q);
    float beta = asinf(fminf(1.0f, fmaxf(-1.0f, r)));
    if (fabsf(beta) + alpha >= kHalfPi) {
        lo = -kQuarterPi;
        hi = kQuarterPi;
        return true;
    }
    float dl = asinf(fminf(1.0f, sinf(alpha) / cosf(beta))) + 1e-5f;
    lo = fmaxf(lam - dl, -kQuarterPi);
    hi = fminf(lam + dl, kQuarterPi);
    return lo <= hi;
}

__device__ inline int cell_index(float angle, int M) {
    float u = tanf(angle);
    return min(M - 1, max(0, int(floorf((u + 1.0f) * 0.5f * M))));
}

// Cell rectangle [iu0, iu1] x [iv0, iv1] of cube face `face` at M x M cells
// that contains every direction within alpha of c on that face.
__device__ inline bool face_cells(float3 c, float alpha, int face, int M, int& iu0, int& iu1, int& iv0, int& iv1) {
    int a = face >> 1;
    float sg = (face & 1) ? -1.0f : 1.0f;
    float comp[3] = {c.x, c.y, c.z};
    float ca = comp[a] * sg, cu = comp[(a + 1) % 3], cv = comp[(a + 2) % 3];
    float ulo, uhi, vlo, vhi;
    if (!lon_range(cu, ca, cv, alpha, ulo, uhi)) return false;
    if (!lon_range(cv, ca, cu, alpha, vlo, vhi)) return false;
    iu0 = cell_index(ulo, M);
    iu1 = cell_index(uhi, M);
    iv0 = cell_index(vlo, M);
    iv1 = cell_index(vhi, M);
    return true;
}

// Stream every candidate of the tile through `fn(rank, valid)` (called by
// all 64 lanes together, one candidate per lane).
template <typename Fn>
__device__ inline void gather_candidates(const SceneView& S, float4 tc0, float4 tc1, int lane, Fn&& fn) {
    if (tc1.z == kCapEmpty || S.n == 0) return;
    float3 c = f3(tc0.x, tc0.y, tc0.z);
    float rho_t = (tc1.z == kCapWide) ? kPi : 2.0f * asinf(fminf(1.0f, tc0.w));
    // lane p: level p / 6, face p % 6
    int p = lane;
    bool has = false;
    int iu0 = 0, iu1 = -1, iv0 = 0, iv1 = -1;
    if (p < 6 * kLevels) {
        int L = p / 6, face = p % 6;
        int M = 1 << L;
        int64_t fb = level_base(L) + int64_t(face) * M * M;
        bool nonempty = S.cell_start[fb] != S.cell_start[fb + int64_t(M) * M];
        if (nonempty) {
            float RL = (L == 0) ? kHalfPi : kQuarterPi / float(M);
            float alpha = rho_t + RL + 1e-5f;
            has = face_cells(c, alpha, face, M, iu0, iu1, iv0, iv1);
        }
    }
    uint64_t todo = __ballot(has);
    while (todo) {
        int q = __ffsll((unsigned long long)todo) - 1;
        todo &= todo - 1;
        int L = q / 6, face = q % 6, M = 1 << L;
        int u0 = __shfl(iu0, q, 64), u1 = __shfl(iu1, q, 64), v0 = __shfl(iv0, q, 64), v1 = __shfl(iv1, q, 64);
        int64_t fb = level_base(L) + int64_t(face) * M * M;
        for (int v = v0; v <= v1; ++v) {
            int64_t c0 = fb + int64_t(v) * M + u0;
            int64_t c1 = fb + int64_t(v) * M + u1;
            uint32_t b = S.cell_start[c0], e = S.cell_start[c1 + 1];
            for (uint32_t k = b; k < e; k += 64) {
                uint32_t idx = k + uint32_t(lane);
                bool valid = idx < e;
                uint32_t rank = valid ? S.cell_list[idx] : 0u;
                fn(rank, valid);
            }
        }
    }
}

__device__ inline bool candidate_test(const SceneView& S, uint32_t rank, float4 tc0, float4 tc1) {
    float4 t0 = S.cap[2 * int64_t(rank)], t1 = S.cap[2 * int64_t(rank) + 1];
    if (t1.z == kCapEmpty) return false;
    const float4* r = S.rec + 4 * int64_t(rank);
    float4 r0 = r[0], r1 = r[1], r2 = r[2];
    return tile_may_see(tc0, tc1, t0, t1, f3(r0.x, r0.y, r0.z), f3(r1.x, r1.y, r1.z), f3(r2.x, r2.y, r2.z));
}

__device__ inline int64_t xcd_remap(int64_t b, int64_t nb) {
    int64_t x = b & 7, loc = b >> 3, q = nb >> 3, r = nb & 7;
    return x * q + (x < r ? x : r) + loc;
}

// ---------------------------------------------------------------- bin ---
// One 256-thread workgroup per 16x16 super-tile (2x2 tiles; wave w owns tile
// w).  The super-tile's cap bounds its four tile caps; the cell rectangles
// of that cap are gathered once, and each candidate is tested against the
// super cap and then against each of the four tile caps.  Survivors are
// appended to the tiles' LDS lists, which are ordered by depth bucket
// (nearest first) and written out.
constexpr int kSupTiles = 4;

struct BinArgs {
    const void* map;
    int64_t ntiles;
    int32_t fmt, depth, lds_cap, all;
    int32_t ntx, nty;
    const void* setup;
    int64_t n;
    void* bins;
    uint32_t* status;  // overflowed-tile counter
};

__device__ inline float4 empty_cap0() { return make_float4(0.f, 0.f, 1.f, 0.f); }
__device__ inline float4 empty_cap1() { return make_float4(1.f, 0.f, kCapEmpty, 0.f); }

// May a triangle (binning record a + unit edge normals) cover a pixel of
// the tile with cap (c0, c1)?  Conservative, like tile_may_see.
__device__ inline bool sub_may_see(float4 c0, float4 c1, float4 a, float3 n0, float3 n1, float3 n2) {
    if (c1.z == kCapEmpty) return false;
    if (c1.z == kCapWide) return true;
    if (a.w < kBinWide) {
        float dx = c0.x - a.x, dy = c0.y - a.y, dz = c0.z - a.z;
        float chord2 = dx * dx + dy * dy + dz * dz;
        float ch_t = sqrtf(fmaxf(0.0f, 1.0f - a.w * a.w));
        float sm = c0.w * ch_t + c1.x * a.w;  // sin((rho_tile + rho_tri)/2)
        if (chord2 > 4.0f * sm * sm * (1.0f + 1e-6f) + 1e-12f) return false;
    }
    float3 c = f3(c0.x, c0.y, c0.z);
    float lim = -c1.y - 1e-6f;
    return !(dot3(n0, c) < lim || dot3(n1, c) < lim || dot3(n2, c) < lim);
}

// Exclusive scan of one value per thread over a 256-thread block.
__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t* s_wsum, uint32_t& total) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) s_wsum[w] = x;
    __syncthreads();
    uint32_t base = 0;
    for (int q = 0; q < w; ++q) base += s_wsum[q];
    total = s_wsum[0] + s_wsum[1] + s_wsum[2] + s_wsum[3];
    __syncthreads();
    return base + x - v;
}

__device__ inline void bin_super(const BinArgs& A, int64_t sidx) {
    extern __shared__ uint32_t lists[];  // kSupTiles x lds_cap
    __shared__ float4 s_cap[kSupTiles][2];
    __shared__ int s_rect[64][4];
    __shared__ uint32_t s_ppre[65];
    __shared__ float4 s_sup[2];
    __shared__ uint32_t s_bk[kSupTiles][kDepthBuckets];
    __shared__ uint32_t s_rb[256], s_pre[256], s_wsum[4], s_cnt[kSupTiles];

    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nsx = (A.ntx + 1) / 2;
    const int sx = int(sidx % nsx), sy = int(sidx / nsx);
    const int tx = 2 * sx + (w & 1), ty = 2 * sy + (w >> 1);
    const bool present = tx < A.ntx && ty < A.nty;
    const int64_t tile = int64_t(ty) * A.ntx + tx;
    const float4* caps = map_caps(A.map, A.ntiles, A.fmt);
    if (lane == 0) {
        s_cap[w][0] = present ? caps[2 * tile] : empty_cap0();
        s_cap[w][1] = present ? caps[2 * tile + 1] : empty_cap1();
    }
    if (tid < kSupTiles) s_cnt[tid] = 0;
    __syncthreads();

    float4 sc0[kSupTiles], sc1[kSupTiles];
#pragma unroll
    for (int q = 0; q < kSupTiles; ++q) {
        sc0[q] = s_cap[q][0];
        sc1[q] = s_cap[q][1];
    }
    // super-tile cap: bounds the four tile caps (computed once, shared)
    if (tid == 0) {
        bool any0 = false, wide0 = false;
        float3 sum = f3(0.f, 0.f, 0.f);
        for (int q = 0; q < kSupTiles; ++q) {
            if (sc1[q].z == kCapEmpty) continue;
            any0 = true;
            if (sc1[q].z == kCapWide) wide0 = true;
            sum = add3(sum, f3(sc0[q].x, sc0[q].y, sc0[q].z));
        }
        float3 c = f3(0.f, 0.f, 1.f);
        float rho = kPi;
        if (any0 && !wide0) {
            float len = sqrtf(dot3(sum, sum));
            if (len > 1e-3f) {
                c = scale3(sum, 1.0f / len);
                rho = 0.0f;
                for (int q = 0; q < kSupTiles; ++q) {
                    if (sc1[q].z == kCapEmpty) continue;
                    float3 d = sub3(c, f3(sc0[q].x, sc0[q].y, sc0[q].z));
                    float ang = 2.0f * asinf(fminf(1.0f, 0.5f * sqrtf(dot3(d, d))));
                    rho = fmaxf(rho, ang + 2.0f * asinf(fminf(1.0f, sc0[q].w)));
                }
                rho = rho * (1.0f + kCapRelMargin) + 1e-6f;
            }
            if (!(rho < kHalfPi)) wide0 = true;
        }
        float sh = 1.0f, ch = 0.0f;
        if (!wide0) sincosf(0.5f * rho, &sh, &ch);
        s_sup[0] = make_float4(c.x, c.y, c.z, rho);
        s_sup[1] = make_float4(sh, ch, any0 ? 1.0f : 0.0f, wide0 ? 1.0f : 0.0f);
    }
    __syncthreads();
    const float4 sup0 = s_sup[0], sup1 = s_sup[1];
    const float3 cs = f3(sup0.x, sup0.y, sup0.z);
    const float rho_s = sup0.w, sh_s = sup1.x, ch_s = sup1.y;
    const bool any = sup1.z != 0.0f, wide = sup1.w != 0.0f;

    SceneView S = scene_view(A.setup, A.n);
    const float4* binrec =
        reinterpret_cast<const float4*>(reinterpret_cast<const char*>(A.setup) + setup_layout(A.n).binrec_off);
    const uint32_t lcap = uint32_t(A.lds_cap);

    auto append = [&](uint32_t mask, uint32_t rank) {
#pragma unroll
        for (int q = 0; q < kSupTiles; ++q) {
            if (mask & (1u << q)) {
                uint32_t pos = atomicAdd(&s_cnt[q], 1u);
                if (pos < lcap) lists[q * lcap + pos] = rank;
            }
        }
    };

    if (any && A.all) {
        uint32_t live_mask = 0;
#pragma unroll
        for (int q = 0; q < kSupTiles; ++q)
            if (sc1[q].z != kCapEmpty) live_mask |= 1u << q;
        for (int64_t k0 = 0; k0 < A.n; k0 += 256) {
            int64_t r = k0 + tid;
            if (r < A.n && S.cap[2 * r + 1].z != kCapEmpty) append(live_mask, uint32_t(r));
        }
    } else if (any) {
        // (level, face) rectangles: lane p of wave 0 handles level p/6, face p%6
        if (tid < 64) {
            int iu0 = 1, iu1 = 0, iv0 = 1, iv1 = 0;
            if (tid < 6 * kLevels) {
                int L = tid / 6, face = tid % 6, M = 1 << L;
                int64_t fb = level_base(L) + int64_t(face) * M * M;
                if (S.cell_start[fb] != S.cell_start[fb + int64_t(M) * M]) {
                    float RL = (L == 0) ? kHalfPi : kQuarterPi / float(M);
                    float alpha = (wide ? kPi : rho_s) + RL + 1e-5f;
                    if (!face_cells(cs, alpha, face, M, iu0, iu1, iv0, iv1)) {
                        iu0 = 1;
                        iu1 = 0;
                    }
                }
            }
            s_rect[tid][0] = iu0;
            s_rect[tid][1] = iu1;
            s_rect[tid][2] = iv0;
            s_rect[tid][3] = iv1;
            // prefix of row counts over the pairs
            uint32_t nr = (iu0 <= iu1) ? uint32_t(iv1 - iv0 + 1) : 0u, x = nr;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                uint32_t y = __shfl_up(x, o, 64);
                if (tid >= o) x += y;
            }
            s_ppre[tid] = x - nr;
            if (tid == 63) s_ppre[64] = x;
        }
        __syncthreads();
        const uint32_t nrows_all = s_ppre[64];
        // all rows of all pairs, 256 at a time: one contiguous run each
        for (uint32_t rb = 0; rb < nrows_all; rb += 256) {
            const uint32_t nb = min(256u, nrows_all - rb);
            uint32_t len = 0;
            if (uint32_t(tid) < nb) {
                uint32_t r = rb + tid;
                int lo = 0, hi = 63;  // pair holding row r: last p with s_ppre[p] <= r
                while (lo < hi) {
                    int mid = (lo + hi + 1) >> 1;
                    if (s_ppre[mid] <= r)
                        lo = mid;
                    else
                        hi = mid - 1;
                }
                const int L = lo / 6, face = lo % 6, M = 1 << L;
                const int64_t row = level_base(L) + int64_t(face) * M * M +
                                    int64_t(s_rect[lo][2] + int(r - s_ppre[lo])) * M;
                uint32_t b = S.cell_start[row + s_rect[lo][0]], e = S.cell_start[row + s_rect[lo][1] + 1];
                s_rb[tid] = b;
                len = e - b;
            }
            uint32_t total;
            uint32_t pre = block_exclusive_scan(len, s_wsum, total);
            s_pre[tid] = pre;
            __syncthreads();
            // candidates, two per thread per pass so their loads overlap
            for (uint32_t k0 = 0; k0 < total; k0 += 512) {
                float4 a[2];
                int64_t idx[2];
                bool valid[2];
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    uint32_t k = k0 + uint32_t(h * 256 + tid);
                    valid[h] = k < total;
                    idx[h] = 0;
                    if (valid[h]) {
                        int lo = 0, hi = int(nb) - 1;  // row holding candidate k
                        while (lo < hi) {
                            int mid = (lo + hi + 1) >> 1;
                            if (s_pre[mid] <= k)
                                lo = mid;
                            else
                                hi = mid - 1;
                        }
                        idx[h] = int64_t(s_rb[lo]) + (k - s_pre[lo]);
                        a[h] = binrec[4 * idx[h]];
                    }
                }
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    if (!valid[h]) continue;
                    bool pass = true;
                    if (!wide && a[h].w < kBinWide) {
                        float dx = cs.x - a[h].x, dy = cs.y - a[h].y, dz = cs.z - a[h].z;
                        float chord2 = dx * dx + dy * dy + dz * dz;
                        float ch_t = sqrtf(fmaxf(0.0f, 1.0f - a[h].w * a[h].w));
                        float sm = sh_s * ch_t + ch_s * a[h].w;
                        pass = chord2 <= 4.0f * sm * sm * (1.0f + 1e-6f) + 1e-12f;
                    }
                    if (pass) {
                        const float4* br = binrec + 4 * idx[h];
                        float4 b4 = br[1], c4 = br[2], d4 = br[3];
                        float3 n0 = f3(b4.x, b4.y, b4.z), n1 = f3(c4.x, c4.y, c4.z), n2 = f3(d4.x, d4.y, d4.z);
                        uint32_t mask = 0;
#pragma unroll
                        for (int q = 0; q < kSupTiles; ++q)
                            if (sub_may_see(sc0[q], sc1[q], a[h], n0, n1, n2)) mask |= 1u << q;
                        if (mask) append(mask, __float_as_uint(b4.w));
                    }
                }
            }
            __syncthreads();
        }
    }
    __syncthreads();

    // Order every tile's list by depth bucket (nearest first) with a
    // counting sort, scattering straight into the output list.
    const uint32_t depth = uint32_t(A.depth);
    const uint32_t cnt = s_cnt[w];
    const bool keep = present && cnt <= depth;
    const uint32_t* my = lists + w * lcap;
    uint32_t* bk = s_bk[w];
    const int shift = bucket_shift(A.n);
    char* bb = reinterpret_cast<char*>(A.bins);
    uint32_t* out = reinterpret_cast<uint32_t*>(bb + 256 + align256(A.ntiles * 4)) + tile * A.depth;
    if (keep) {
        for (int q = lane; q < kDepthBuckets; q += 64) bk[q] = 0;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        for (uint32_t i = lane; i < cnt; i += 64) atomicAdd(&bk[my[i] >> shift], 1u);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        // exclusive scan of the 256 bucket counts: 4 per lane
        uint32_t c4[4], run = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            c4[q] = bk[4 * lane + q];
            run += c4[q];
        }
        uint32_t x = run;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            uint32_t y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        uint32_t base = x - run;
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            bk[4 * lane + q] = base;
            base += c4[q];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        for (uint32_t i = lane; i < cnt; i += 64) {
            uint32_t r = my[i];
            out[atomicAdd(&bk[r >> shift], 1u)] = r;
        }
    }
    if (present) {
        uint32_t* counts = reinterpret_cast<uint32_t*>(bb + 256);
        if (lane == 0) {
            counts[tile] = cnt;
            if (!keep) atomicAdd(A.status, 1u);
        }
    }
}

__global__ __launch_bounds__(256) void k_bin(BinArgs A) { bin_super(A, xcd_remap(blockIdx.x, gridDim.x)); }

__global__ __launch_bounds__(64) void k_zero_u32(uint32_t* p, int64_t n) {
    int64_t i = int64_t(blockIdx.x) * 64 + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// ------------------------------------------------------------- raster ---
struct RasterArgs {
    const void* map;
    int64_t ntiles;
    int32_t fmt, depth, W, H, ntx, pad;
    const void* setup;
    int64_t n;
    const void* bins;
    uint32_t* tri_id;
    float* out_depth;
    unsigned long long* stats;  // instrumented variant only: tests, covered, triangles, tiles
    int32_t no_early_exit;      // instrumented variant only: process whole lists
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

template <bool kStats>
__device__ inline void raster_tile(const RasterArgs& A, int64_t tile, int lane) {
    const float4* caps = map_caps(A.map, A.ntiles, A.fmt);
    SceneView S = scene_view(A.setup, A.n);
    const char* bb = reinterpret_cast<const char*>(A.bins);
    const uint32_t* counts = reinterpret_cast<const uint32_t*>(bb + 256);
    const uint32_t* lists = reinterpret_cast<const uint32_t*>(bb + 256 + align256(A.ntiles * 4));

    int tx = int(tile % A.ntx), ty = int(tile / A.ntx);
    int i = tx * kTile + (lane & (kTile - 1)), j = ty * kTile + (lane >> 3);
    bool inside = i < A.W && j < A.H;
    float3 g = load_dir(A.map, A.fmt, A.ntiles, tile, lane);
    bool has_dir = inside && (g.x != 0.0f || g.y != 0.0f || g.z != 0.0f);
    uint64_t best = kKeyEmpty;
    uint32_t count = counts[tile];
    unsigned long long n_tri = 0, n_cov = 0;
    if (count <= uint32_t(A.depth)) {
        // Records are fetched 16 at a time: lane l loads float4 (l & 3) of
        // triangle (l >> 2) of the group, one vector load for the whole
        // wave, staged in LDS and read back as broadcasts.  The next group's
        // records and the group after's ranks are in flight meanwhile.
        __shared__ float4 s_stage[4][64];
        float4* stg = s_stage[threadIdx.x >> 6];
        const uint32_t* lst = lists + tile * A.depth;
        const float4* rec = S.rec;
        const uint32_t ngroups = (count + 15u) >> 4;
        const uint32_t sub = uint32_t(lane) >> 2, part = uint32_t(lane) & 3u;
        uint32_t rk = sub < count ? lst[sub] : 0u;
        float4 v = rec[4 * int64_t(rk) + part];
        rk = 16u + sub < count ? lst[16u + sub] : 0u;
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
            for (uint32_t t8 = 0; t8 < nt; t8 += 8) {
                if (!(kStats && A.no_early_exit)) {
                    // nearest-first early exit: every pixel already beats the
                    // depth lower bound of this triangle's bucket, which bounds
                    // every triangle still to come
                    float lb = __builtin_amdgcn_readfirstlane(stg[4 * t8 + 3].w);
                    uint32_t worst = wave_max_u32_dpp(has_dir ? uint32_t(best >> 32) : 0u);
                    if (lb > __uint_as_float(worst)) {
                        done = true;
                        break;
                    }
                }
#pragma unroll
                for (uint32_t u = 0; u < 8; ++u) {
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
    } else {
        float4 tc0 = caps[2 * tile], tc1 = caps[2 * tile + 1];
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

template <bool kStats>
__global__ __launch_bounds__(256) void k_raster(RasterArgs A) {
    int w = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    int64_t tile = xcd_remap(blockIdx.x, gridDim.x) * 4 + w;
    if (tile >= A.ntiles) return;
    raster_tile<kStats>(A, tile, threadIdx.x & 63);
}

// ------------------------------------------------------------ launchers --
int32_t bin_lds_cap(int32_t depth) {
    int32_t c = 64;
    while (c < depth) c <<= 1;
    return c;
}

int64_t bin_grid(int32_t ntx, int32_t nty) { return int64_t((ntx + 1) / 2) * ((nty + 1) / 2); }

hipError_t launch_bin(const void* map, int32_t W, int32_t H, int32_t fmt, const void* setup, int64_t n, int32_t depth,
                      bool all, void* bins, hipStream_t st) {
    MapLayout ML = map_layout(W, H, fmt);
    BinArgs A;
    A.map = map;
    A.ntiles = ML.ntiles;
    A.fmt = fmt;
    A.depth = depth;
    A.lds_cap = bin_lds_cap(depth);
    A.all = all ? 1 : 0;
    A.ntx = ML.ntx;
    A.nty = ML.nty;
    A.setup = setup;
    A.n = n;
    A.bins = bins;
    A.status = reinterpret_cast<uint32_t*>(bins);
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, reinterpret_cast<uint32_t*>(bins), int64_t(64));
    hipLaunchKernelGGL(k_bin, dim3(unsigned(bin_grid(ML.ntx, ML.nty))), dim3(256),
                       size_t(kSupTiles) * A.lds_cap * 4, st, A);
    return hipGetLastError();
}

hipError_t launch_raster(const void* map, int32_t W, int32_t H, int32_t fmt, const void* setup, int64_t n,
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
    A.pad = 0;
    A.setup = setup;
    A.n = n;
    A.bins = bins;
    A.tri_id = tri_id;
    A.out_depth = out_depth;
    A.stats = stats;
    A.no_early_exit = no_early_exit;
    int64_t blocks = (ML.ntiles + 3) / 4;
    if (stats) {
        hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, reinterpret_cast<uint32_t*>(stats), int64_t(8));
        hipLaunchKernelGGL(k_raster<true>, dim3(unsigned(blocks)), dim3(256), 0, st, A);
    } else {
        hipLaunchKernelGGL(k_raster<false>, dim3(unsigned(blocks)), dim3(256), 0, st, A);
    }
    return hipGetLastError();
}

}  // namespace vsr
