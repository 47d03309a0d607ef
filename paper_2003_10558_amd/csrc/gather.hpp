// Candidate gathering from the setup's cube-map cap index.
//
// A tile's cap (centre c, radius rho) can only meet the cap of a triangle
// filed at index level L (cap radius <= R_L = (pi/4)/2^L, level 0: pi/2) if
// the triangle's cap centre lies within rho + R_L of c.  For every level and
// cube face the rectangle of cells that such centres can occupy follows from
// the longitude/latitude extent of a spherical cap; every row of that
// rectangle is one contiguous run of the (slice, cell)-sorted triangle list.
// Candidates are then tested conservatively (caps and edge planes, with
// margins far above FP32 rounding) so that a (tile, triangle) pair the
// rasterizer could cover is never dropped.
//
// Two gatherers share this machinery:
//   gather_candidates  one wavefront, one tile (the rasterizer's fallback
//                      for tiles whose bin overflowed);
//   gather_slices      one 256-thread workgroup, one 16x16 super-tile of four
//                      tiles, a range of depth slices, candidates streamed
//                      through all threads (binning and the fused renderer).
#pragma once
#include "vsr_internal.h"

namespace vsr {

struct SceneView {
    const float4* rec;         // 4 x float4 per triangle, nearest-first (rank) order
    const float4* cap;         // 2 x float4 per triangle, rank order
    const uint32_t* cell_list; // ranks sorted by (slice, cell)
    const uint32_t* cell_start;
    const float4* binrec;      // cell-ordered binning records
    const uint32_t* face_count;
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
    s.binrec = reinterpret_cast<const float4*>(b + L.binrec_off);
    s.face_count = reinterpret_cast<const uint32_t*>(b + L.face_count_off);
    s.n = n;
    return s;
}

// Longitude range of a cap (centre with components p along the measured
// axis, q along the face normal, r along the rotation axis; radius alpha),
// intersected with the face's [-pi/4, pi/4], as u = tan(longitude).  False
// when empty.  General, for caps that reach the face's plane.
__device__ inline bool lon_range(float p, float q, float r, float alpha, float& lo, float& hi) {
    float lam = atan2f(p, q);
    float beta = asinf(fminf(1.0f, fmaxf(-1.0f, r)));
    if (fabsf(beta) + alpha >= kHalfPi) {
        lo = -1.0f;
        hi = 1.0f;
        return true;
    }
    float dl = asinf(fminf(1.0f, sinf(alpha) / cosf(beta))) + 1e-5f;
    float a = fmaxf(lam - dl, -kQuarterPi), b = fminf(lam + dl, kQuarterPi);
    if (a > b) return false;
    lo = tanf(a);
    hi = tanf(b);
    return true;
}

// Range of u = p_u / p_a over a cap (centre c, sa = sine of its radius)
// lying wholly in the half-space p_a > 0 (ca > sa), clipped to [-1, 1]; the
// extremes are where a plane p_u = u p_a through O is tangent to the cap:
// (cu - u ca)^2 = sa^2 (1 + u^2).  False when the range misses [-1, 1].
__device__ inline bool tangent_range(float ca, float cu, float sa, float& lo, float& hi) {
    const float den = ca * ca - sa * sa;
    const float root = sa * sqrtf(fmaxf(0.0f, ca * ca + cu * cu - sa * sa));
    const float mid = ca * cu;
    const float u1 = (mid - root) / den, u2 = (mid + root) / den;
    lo = fmaxf(u1 - 1e-5f * (1.0f + fabsf(u1)), -1.0f);
    hi = fminf(u2 + 1e-5f * (1.0f + fabsf(u2)), 1.0f);
    return lo <= hi;
}

__device__ inline int cell_index(float u, int M) {
    return min(M - 1, max(0, int(floorf((u + 1.0f) * 0.5f * M))));
}

// Angle from a cube face's centre axis to its corners, acos(1/sqrt(3)), plus
// a margin: the face lies inside the cap of this radius around its axis.
constexpr float kFaceRadius = 0.95533f;
constexpr float kCosFace = 0.5773390f;  // cos(kFaceRadius) = 0.57733934..., rounded down
constexpr float kSinFace = 0.8165046f;  // sin(kFaceRadius) = 0.81650431..., rounded up

// face_cells with the cap radius given by its sine and cosine (sa, ca_):
// no transcendental on the common path.
__device__ inline bool face_cells_sc(float3 c, float sa, float ca_, int face, int M, int& iu0, int& iu1, int& iv0,
                                     int& iv1) {
    if (!(ca_ > 0.0f)) {  // radius >= pi/2
        iu0 = iv0 = 0;
        iu1 = iv1 = M - 1;
        return true;
    }
    const int a = face >> 1;
    const float sg = (face & 1) ? -1.0f : 1.0f;
    const float comp[3] = {c.x, c.y, c.z};
    const float cax = comp[a] * sg, cu = comp[(a + 1) % 3], cv = comp[(a + 2) % 3];
    // reject faces outside the cap of radius alpha + kFaceRadius around c
    const float cf = ca_ * kCosFace - sa * kSinFace;  // cos(alpha + face radius)
    const float sf = sa * kCosFace + ca_ * kSinFace;
    if (sf > 0.0f && cax < cf - 1e-6f) return false;
    float ulo, uhi, vlo, vhi;
    if (cax > sa * (1.0f + 1e-5f) + 1e-6f) {
        if (!tangent_range(cax, cu, sa, ulo, uhi)) return false;
        if (!tangent_range(cax, cv, sa, vlo, vhi)) return false;
    } else {
        const float alpha = atan2f(sa, ca_);
        if (!lon_range(cu, cax, cv, alpha, ulo, uhi)) return false;
        if (!lon_range(cv, cax, cu, alpha, vlo, vhi)) return false;
    }
    iu0 = cell_index(ulo, M);
    iu1 = cell_index(uhi, M);
    iv0 = cell_index(vlo, M);
    iv1 = cell_index(vhi, M);
    return true;
}

// Cell rectangle [iu0, iu1] x [iv0, iv1] of cube face `face` at M x M cells
// that contains every direction within alpha of c on that face.
__device__ inline bool face_cells(float3 c, float alpha, int face, int M, int& iu0, int& iu1, int& iv0, int& iv1) {
    if (!(alpha < kHalfPi)) {
        iu0 = iv0 = 0;
        iu1 = iv1 = M - 1;
        return true;
    }
    const int a = face >> 1;
    const float sg = (face & 1) ? -1.0f : 1.0f;
    const float comp[3] = {c.x, c.y, c.z};
    const float ca = comp[a] * sg, cu = comp[(a + 1) % 3], cv = comp[(a + 2) % 3];
    if (alpha + kFaceRadius < kPi && ca < cosf(alpha + kFaceRadius + 1e-5f)) return false;
    float ulo, uhi, vlo, vhi;
    const float sa = sinf(alpha);
    if (ca > sa * (1.0f + 1e-5f) + 1e-6f) {
        if (!tangent_range(ca, cu, sa, ulo, uhi)) return false;
        if (!tangent_range(ca, cv, sa, vlo, vhi)) return false;
    } else {
        if (!lon_range(cu, ca, cv, alpha, ulo, uhi)) return false;
        if (!lon_range(cv, ca, cu, alpha, vlo, vhi)) return false;
    }
    iu0 = cell_index(ulo, M);
    iu1 = cell_index(uhi, M);
    iv0 = cell_index(vlo, M);
    iv1 = cell_index(vhi, M);
    return true;
}

__device__ inline int64_t xcd_remap(int64_t b, int64_t nb) {
    int64_t x = b & 7, loc = b >> 3, q = nb >> 3, r = nb & 7;
    return x * q + (x < r ? x : r) + loc;
}

__device__ inline float4 empty_cap0() { return make_float4(0.f, 0.f, 1.f, 0.f); }
__device__ inline float4 empty_cap1() { return make_float4(1.f, 0.f, kCapEmpty, 0.f); }

// May a triangle (binning record a + unit edge normals) cover a pixel of
// the tile with cap (c0, c1)?  Never false for a pair the rasterizer's FP32
// test could cover.
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

// ---------------------------------------------------- one wave, one tile --

// Stream every candidate of the tile, all slices, through fn(rank, valid)
// (called by all 64 lanes together, one candidate per lane).
template <typename Fn>
__device__ inline void gather_candidates(const SceneView& S, float4 tc0, float4 tc1, int lane, Fn&& fn) {
    if (tc1.z == kCapEmpty || S.n == 0) return;
    float3 c = f3(tc0.x, tc0.y, tc0.z);
    float rho_t = (tc1.z == kCapWide) ? kPi : 2.0f * asinf(fminf(1.0f, tc0.w));
    bool has = false;
    int iu0 = 0, iu1 = -1, iv0 = 0, iv1 = -1;
    if (lane < 6 * kLevels) {
        int L = lane / 6, face = lane % 6, M = 1 << L;
        float RL = (L == 0) ? kHalfPi : kQuarterPi / float(M);
        has = face_cells(c, rho_t + RL + 1e-5f, face, M, iu0, iu1, iv0, iv1);
    }
    uint64_t todo = __ballot(has);
    while (todo) {
        int q = __ffsll((unsigned long long)todo) - 1;
        todo &= todo - 1;
        int L = q / 6, face = q % 6, M = 1 << L;
        int u0 = __shfl(iu0, q, 64), u1 = __shfl(iu1, q, 64), v0 = __shfl(iv0, q, 64), v1 = __shfl(iv1, q, 64);
        for (int s = 0; s < kSlices; ++s) {
            if (S.face_count[s * 64 + q] == 0) continue;
            int64_t fb = int64_t(s) * kNumBuckets + level_base(L) + int64_t(face) * M * M;
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
}

__device__ inline bool candidate_test(const SceneView& S, uint32_t rank, float4 tc0, float4 tc1) {
    float4 t0 = S.cap[2 * int64_t(rank)], t1 = S.cap[2 * int64_t(rank) + 1];
    if (t1.z == kCapEmpty) return false;
    const float4* r = S.rec + 4 * int64_t(rank);
    float4 r0 = r[0], r1 = r[1], r2 = r[2];
    return tile_may_see(tc0, tc1, t0, t1, f3(r0.x, r0.y, r0.z), f3(r1.x, r1.y, r1.z), f3(r2.x, r2.y, r2.z));
}

// ------------------------------------------- one workgroup, 4 tiles -----

constexpr int kSupTiles = 4;

struct SuperShared {
    float4 cap[kSupTiles][2];
    float4 sup[2];
    int rect[64][4];
    uint32_t ppre[65];
    uint32_t spre[64][kSlices + 1];
    uint32_t rb[256], pre[256], wsum[4];
    uint32_t cnt[kSupTiles];
    uint32_t flag[kSupTiles];
    uint32_t fc[kSlices * 64];  // per-slice (level, face) triangle counts
    uint32_t bk[kSupTiles][kDepthBuckets];
};
static_assert(kSlices * 64 == 256, "one face count per thread of the 256-thread block");

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

// Tile of wave w in super-tile sidx (2x2 tiles); false when outside the map.
__device__ inline bool super_tile_of(int64_t sidx, int w, int ntx, int nty, int64_t& tile, int& tx, int& ty) {
    const int nsx = (ntx + 1) / 2;
    const int sx = int(sidx % nsx), sy = int(sidx / nsx);
    tx = 2 * sx + (w & 1);
    ty = 2 * sy + (w >> 1);
    tile = int64_t(ty) * ntx + tx;
    return tx < ntx && ty < nty;
}

// Loads the four tile caps and the per-slice face counts, computes the
// super-tile cap and the cell rectangles of every (level, face).  All
// threads of the block call it.  Angles are never formed: caps carry
// sin and cos of their half radius, and radii add through the angle-sum
// identities.
__device__ inline void super_setup(SuperShared& sh, const float4* caps, const uint32_t* face_count, bool present,
                                   int64_t tile) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    if (lane == 0) {
        sh.cap[w][0] = present ? caps[2 * tile] : empty_cap0();
        sh.cap[w][1] = present ? caps[2 * tile + 1] : empty_cap1();
    }
    sh.fc[tid] = face_count[tid];  // kSlices * 64 == 256 entries
    if (tid < kSupTiles) {
        sh.cnt[tid] = 0;
        sh.flag[tid] = 0;
    }
    __syncthreads();
    if (tid == 0) {
        bool any0 = false, wide0 = false;
        float3 sum = f3(0.f, 0.f, 0.f);
        for (int q = 0; q < kSupTiles; ++q) {
            float4 c0 = sh.cap[q][0], c1 = sh.cap[q][1];
            if (c1.z == kCapEmpty) continue;
            any0 = true;
            if (c1.z == kCapWide) wide0 = true;
            sum = add3(sum, f3(c0.x, c0.y, c0.z));
        }
        float3 c = f3(0.f, 0.f, 1.f);
        float sh_ = 1.0f, ch_ = 0.0f;  // sin, cos of half the super-cap radius
        if (any0 && !wide0) {
            float len = sqrtf(dot3(sum, sum));
            if (len > 1e-3f) {
                c = scale3(sum, 1.0f / len);
                sh_ = 0.0f;
                ch_ = 1.0f;
                for (int q = 0; q < kSupTiles; ++q) {
                    float4 c0 = sh.cap[q][0], c1 = sh.cap[q][1];
                    if (c1.z == kCapEmpty) continue;
                    // half-angle between the centres from the chord, plus the
                    // tile's half radius: sin/cos of the sum
                    float3 d = sub3(c, f3(c0.x, c0.y, c0.z));
                    float st = fminf(1.0f, 0.5f * sqrtf(dot3(d, d)));
                    float ct = sqrtf(fmaxf(0.0f, 1.0f - st * st));
                    float sq = st * c1.x + ct * c0.w, cq = ct * c1.x - st * c0.w;
                    if (!(cq > 0.0f)) {
                        wide0 = true;
                    } else if (sq > sh_) {
                        sh_ = sq;
                        ch_ = cq;
                    }
                }
                // margin: grow the half radius by a relative 1e-6 and 1e-7 rad
                sh_ = sh_ * (1.0f + 1e-6f) + 1e-7f;
                ch_ = sqrtf(fmaxf(0.0f, 1.0f - sh_ * sh_));
            } else {
                wide0 = true;
            }
            if (!(sh_ < 0.70710678f)) wide0 = true;  // radius >= pi/2
        }
        if (wide0) {
            sh_ = 1.0f;
            ch_ = 0.0f;
        }
        sh.sup[0] = make_float4(c.x, c.y, c.z, sh_);
        sh.sup[1] = make_float4(sh_, ch_, any0 ? 1.0f : 0.0f, wide0 ? 1.0f : 0.0f);
    }
    __syncthreads();
    if (tid < 64) {
        const float4 sup0 = sh.sup[0], sup1 = sh.sup[1];
        int iu0 = 1, iu1 = 0, iv0 = 1, iv1 = 0;
        if (tid < 6 * kLevels && sup1.z != 0.0f) {
            const int L = tid / 6, face = tid % 6, M = 1 << L;
            const float RL = ((L == 0) ? kHalfPi : kQuarterPi / float(M)) + 1e-5f;
            if (sup1.w != 0.0f) {
                iu0 = iv0 = 0;
                iu1 = iv1 = M - 1;
            } else {
                // alpha = super radius + R_L: sin and cos from the sum identities
                const float srho = 2.0f * sup1.x * sup1.y, crho = 1.0f - 2.0f * sup1.x * sup1.x;
                float sR, cR;
                sincosf(RL, &sR, &cR);
                const float sa = srho * cR + crho * sR, ca = crho * cR - srho * sR;
                if (!face_cells_sc(f3(sup0.x, sup0.y, sup0.z), sa, ca, face, M, iu0, iu1, iv0, iv1)) {
                    iu0 = 1;
                    iu1 = 0;
                }
            }
        }
        sh.rect[tid][0] = iu0;
        sh.rect[tid][1] = iu1;
        sh.rect[tid][2] = iv0;
        sh.rect[tid][3] = iv1;
    }
    __syncthreads();
}

// Streams the candidates of depth slices [s0, s1) through the super-tile
// tests.  The rows of every (level, face, slice) are flattened into one
// list so that their cell ranges load and scan in one pass.
// append(mask, rank) receives every survivor with the set of tiles (bits of
// live_mask) it may cover; chunk_end() runs after every 256 candidates, by
// all threads (a point where the caller may synchronise).  All threads of
// the block call this with the same arguments.
template <typename Append, typename ChunkEnd>
__device__ inline void gather_slices(SuperShared& sh, const SceneView& S, int s0, int s1, uint32_t live_mask,
                                     Append&& append, ChunkEnd&& chunk_end) {
    const int tid = threadIdx.x;
    const float4 sup0 = sh.sup[0], sup1 = sh.sup[1];
    const float3 cs = f3(sup0.x, sup0.y, sup0.z);
    const float sh_s = sup1.x, ch_s = sup1.y;
    const bool wide = sup1.w != 0.0f;
    if (tid < 64) {
        // rows of pair `tid`, slice-major over the slices that have triangles
        const int iu0 = sh.rect[tid][0], iu1 = sh.rect[tid][1], iv0 = sh.rect[tid][2], iv1 = sh.rect[tid][3];
        const uint32_t rows = (tid < 6 * kLevels && iu0 <= iu1) ? uint32_t(iv1 - iv0 + 1) : 0u;
        uint32_t nr = 0;
        for (int s = s0; s < s1; ++s) {
            sh.spre[tid][s - s0] = nr;
            if (rows && sh.fc[s * 64 + tid] != 0) nr += rows;
        }
        sh.spre[tid][s1 - s0] = nr;
        uint32_t x = nr;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            uint32_t y = __shfl_up(x, o, 64);
            if (tid >= o) x += y;
        }
        sh.ppre[tid] = x - nr;
        if (tid == 63) sh.ppre[64] = x;
    }
    __syncthreads();
    float4 tc0[kSupTiles], tc1[kSupTiles];
#pragma unroll
    for (int q = 0; q < kSupTiles; ++q) {
        tc0[q] = sh.cap[q][0];
        tc1[q] = sh.cap[q][1];
    }
    const uint32_t nrows_all = sh.ppre[64];
    for (uint32_t rb = 0; rb < nrows_all; rb += 256) {
        const uint32_t nb = min(256u, nrows_all - rb);
        uint32_t len = 0;
        if (uint32_t(tid) < nb) {
            const uint32_t r = rb + tid;
            int lo = 0, hi = 63;  // (level, face) holding row r: last p with ppre[p] <= r
            while (lo < hi) {
                int mid = (lo + hi + 1) >> 1;
                if (sh.ppre[mid] <= r)
                    lo = mid;
                else
                    hi = mid - 1;
            }
            const uint32_t rl = r - sh.ppre[lo];
            int sl = 0;  // slice within the pair: last with spre <= rl
            while (sl + 1 < s1 - s0 && sh.spre[lo][sl + 1] <= rl) ++sl;
            const int L = lo / 6, face = lo % 6, M = 1 << L;
            const int64_t row = int64_t(s0 + sl) * kNumBuckets + level_base(L) + int64_t(face) * M * M +
                                int64_t(sh.rect[lo][2] + int(rl - sh.spre[lo][sl])) * M;
            uint32_t b = S.cell_start[row + sh.rect[lo][0]], e = S.cell_start[row + sh.rect[lo][1] + 1];
            sh.rb[tid] = b;
            len = e - b;
        }
        uint32_t total;
        uint32_t pre = block_exclusive_scan(len, sh.wsum, total);
        sh.pre[tid] = pre;
        __syncthreads();
        for (uint32_t k0 = 0; k0 < total; k0 += 256) {
            uint32_t k = k0 + uint32_t(tid);
            if (k < total) {
                int lo = 0, hi = int(nb) - 1;  // row holding candidate k
                while (lo < hi) {
                    int mid = (lo + hi + 1) >> 1;
                    if (sh.pre[mid] <= k)
                        lo = mid;
                    else
                        hi = mid - 1;
                }
                const float4* br = S.binrec + 4 * (int64_t(sh.rb[lo]) + (k - sh.pre[lo]));
                float4 a = br[0];
                bool pass = true;
                if (!wide && a.w < kBinWide) {
                    float dx = cs.x - a.x, dy = cs.y - a.y, dz = cs.z - a.z;
                    float chord2 = dx * dx + dy * dy + dz * dz;
                    float ch_t = sqrtf(fmaxf(0.0f, 1.0f - a.w * a.w));
                    float sm = sh_s * ch_t + ch_s * a.w;
                    pass = chord2 <= 4.0f * sm * sm * (1.0f + 1e-6f) + 1e-12f;
                }
                if (pass) {
                    float4 b4 = br[1], c4 = br[2], d4 = br[3];
                    float3 n0 = f3(b4.x, b4.y, b4.z), n1 = f3(c4.x, c4.y, c4.z), n2 = f3(d4.x, d4.y, d4.z);
                    uint32_t mask = 0;
#pragma unroll
                    for (int q = 0; q < kSupTiles; ++q)
                        if ((live_mask >> q) & 1u)
                            if (sub_may_see(tc0[q], tc1[q], a, n0, n1, n2)) mask |= 1u << q;
                    if (mask) append(mask, __float_as_uint(b4.w));
                }
            }
            chunk_end();
        }
        __syncthreads();
    }
}

// Counting sort of one wave's list (ranks) by depth bucket into `out`.
__device__ inline void bucket_sort_wave(const uint32_t* in, uint32_t cnt, uint32_t* bk, int shift, uint32_t* out) {
    const int lane = threadIdx.x & 63;
    for (int q = lane; q < kDepthBuckets; q += 64) bk[q] = 0;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    for (uint32_t i = lane; i < cnt; i += 64) atomicAdd(&bk[in[i] >> shift], 1u);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
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
        uint32_t r = in[i];
        out[atomicAdd(&bk[r >> shift], 1u)] = r;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

}  // namespace vsr
