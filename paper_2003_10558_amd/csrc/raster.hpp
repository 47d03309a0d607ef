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
// Binning keeps the survivors in LDS, sorts them (they are triangle ranks,
// i.e. nearest-first order) with a bitonic network and writes the tile's
// list.
//
// Rasterization: each lane owns one pixel direction g and a 64-bit z-buffer
// key (depth bits << 32 | triangle id).  For every listed triangle, read
// with wave-uniform scalar loads, the lane forms the three oriented
// edge-plane values n_i . g (section 1.1); all three > 0 is the binary step
// of section 1.1.1.  Covered lanes take r = d / (g . N) (section 1.1.4) and
// keep the smaller key (depth-pass test, section 1.4; ties to the lower id).
// Lists are nearest first: once every pixel of the tile holds a depth below
// the next triangle's depth lower bound, no later triangle can win and the
// wave stops.
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
struct BinArgs {
    const void* map;
    int64_t ntiles;
    int32_t fmt, depth, lds_cap, all;
    const void* setup;
    int64_t n;
    void* bins;
    uint32_t* status;  // overflowed-tile counter
};

__device__ inline void bin_tile(const BinArgs& A, int64_t tile, int lane, uint32_t* lst) {
    const float4* caps = map_caps(A.map, A.ntiles, A.fmt);
    float4 tc0 = caps[2 * tile], tc1 = caps[2 * tile + 1];
    SceneView S = scene_view(A.setup, A.n);
    char* bb = reinterpret_cast<char*>(A.bins);
    uint32_t* counts = reinterpret_cast<uint32_t*>(bb + 256);
    uint32_t* lists = reinterpret_cast<uint32_t*>(bb + 256 + align256(A.ntiles * 4));
    uint32_t count = 0;
    const uint32_t cap_n = uint32_t(A.lds_cap);
    auto push = [&](uint32_t rank, bool pass) {
        uint64_t m = __ballot(pass);
        uint32_t pos = count + __builtin_amdgcn_mbcnt_hi(uint32_t(m >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(m), 0u));
        if (pass && pos < cap_n) lst[pos] = rank;
        count += uint32_t(__popcll(m));
    };
    if (A.all) {
        if (tc1.z != kCapEmpty) {
            for (int64_t k = 0; k < A.n; k += 64) {
                int64_t idx = k + lane;
                bool valid = idx < A.n;
                bool pass = valid && S.cap[2 * idx + 1].z != kCapEmpty;
                push(uint32_t(idx), pass);
            }
        }
    } else {
        gather_candidates(S, tc0, tc1, lane, [&](uint32_t rank, bool valid) {
            bool pass = valid && candidate_test(S, rank, tc0, tc1);
            push(rank, pass);
        });
    }
    __syncthreads();
    if (count <= uint32_t(A.depth)) {
        // bitonic sort of the first count entries, padded to a power of two
        uint32_t np = 1;
        while (np < count) np <<= 1;
        for (uint32_t i = count + lane; i < np; i += 64) lst[i] = 0xFFFFFFFFu;
        __syncthreads();
        for (uint32_t k = 2; k <= np; k <<= 1) {
            for (uint32_t j = k >> 1; j > 0; j >>= 1) {
                for (uint32_t i = lane; i < np; i += 64) {
                    uint32_t l = i ^ j;
                    if (l > i) {
                        uint32_t a = lst[i], b = lst[l];
                        bool up = (i & k) == 0;
                        if ((a > b) == up) {
                            lst[i] = b;
                            lst[l] = a;
                        }
                    }
                }
                __syncthreads();
            }
        }
        uint32_t* out = lists + tile * A.depth;
        for (uint32_t i = lane; i < count; i += 64) out[i] = lst[i];
    } else if (lane == 0) {
        atomicAdd(A.status, 1u);  // overflowed tiles
    }
    if (lane == 0) counts[tile] = count;
}

__global__ __launch_bounds__(64) void k_bin(BinArgs A) {
    extern __shared__ uint32_t lst[];
    int64_t tile = xcd_remap(blockIdx.x, gridDim.x);
    bin_tile(A, tile, threadIdx.x, lst);
}

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

// One triangle against the lane's pixel; returns whether it covers it.
__device__ inline bool raster_one(const float4* __restrict__ rec, uint32_t rank, float3 g, uint64_t& best) {
    const float4* r = rec + 4 * int64_t(rank);
    float4 r0 = r[0], r1 = r[1], r2 = r[2], r3 = r[3];
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
        const uint32_t* lst = lists + tile * A.depth;
        for (uint32_t k = 0; k < count; ++k) {
            uint32_t rank = lst[k];
            if ((k & 7u) == 0u && !(kStats && A.no_early_exit)) {
                // nearest-first early exit: every pixel already beats the
                // next triangle's depth lower bound
                uint32_t worst = __builtin_amdgcn_readfirstlane(wave_max_u32(has_dir ? uint32_t(best >> 32) : 0u));
                float lb = S.rec[4 * int64_t(rank) + 3].y;
                if (lb > __uint_as_float(worst)) break;
            }
            bool cov = raster_one(S.rec, rank, g, best);
            if (kStats) {
                n_tri += 1;
                n_cov += __popcll(__ballot(cov));
            }
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
    if (kStats && lane == 0) {
        atomicAdd(&A.stats[0], n_tri * (unsigned long long)__popcll(__ballot(has_dir)));
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
    while (c < depth + 1) c <<= 1;  // room for depth+1 entries detects overflow
    return c;
}

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
    A.setup = setup;
    A.n = n;
    A.bins = bins;
    A.status = reinterpret_cast<uint32_t*>(bins);
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, reinterpret_cast<uint32_t*>(bins), int64_t(64));
    hipLaunchKernelGGL(k_bin, dim3(unsigned(ML.ntiles)), dim3(64), size_t(A.lds_cap) * 4, st, A);
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
