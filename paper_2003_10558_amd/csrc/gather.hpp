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
//   gather_slices      one 256-thread workgroup, one gathering cap (a 16x16
//                      super-tile or a 32x32 block), a range of depth
//                      slices, candidates streamed through all threads
//                      (both binner shapes and the fused renderer).
#pragma once
#include "vsr_internal.h"

namespace vsr {

struct SceneView {
    const float4* rec;         // 4 x float4 per triangle, nearest-first (rank) order
    const float4* cap;         // 2 x float4 per triangle, rank order
    const float4* rcap;        // binning cap (as bincap) per triangle, rank order
    const uint32_t* cell_list; // ranks sorted by (slice, cell)
    const uint32_t* cell_start;
    const float4* bincap;      // cell-ordered caps: centre, sine of half radius (kBinWide: wide)
    const float4* binnrm;      // cell-ordered unit edge normals (3 per triangle; rank in .w of the first)
    const uint32_t* face_count;
    int64_t n;
};

__device__ inline SceneView scene_view(const void* setup, int64_t n) {
    SetupLayout L = setup_layout(n);
    const char* b = reinterpret_cast<const char*>(setup);
    SceneView s;
    s.rec = reinterpret_cast<const float4*>(b + L.rec_off);
    s.cap = reinterpret_cast<const float4*>(b + L.cap_off);
    s.rcap = reinterpret_cast<const float4*>(b + L.rcap_off);
    s.cell_list = reinterpret_cast<const uint32_t*>(b + L.cell_list_off);
    s.cell_start = reinterpret_cast<const uint32_t*>(b + L.cell_start_off);
    s.bincap = reinterpret_cast<const float4*>(b + L.bincap_off);
    s.binnrm = reinterpret_cast<const float4*>(b + L.binnrm_off);
    s.face_count = reinterpret_cast<const uint32_t*>(b + L.face_count_off);
    s.n = n;
    return s;
}

// Range of u = p_u / p_a, clipped to [-1, 1], over the directions p of a cap
// that lie on the cube face with axis a.  The cap has centre components ca
// (along a) and cu (along u) and radius alpha < pi/2 with sine sa.  Such a p
// lies on the plane through O on which p_u = u p_a; the centre is then within
// alpha of that plane, |cu - u ca| <= sa sqrt(1 + u^2), i.e.
//   f(u) = (ca^2 - sa^2) u^2 - 2 ca cu u + cu^2 - sa^2 <= 0.
// The hull of {u in [-1, 1] : f(u) <= 0} in FP32, each root widened by a
// bound on its rounding error (u = 2^-24; den = ca^2 - sa^2 and
// disc = ca^2 + cu^2 - sa^2 carry at most 3u (ca^2 + sa^2) and 9u, the
// numerator mid +- root 2u (|mid| + root) plus the square root's
// 9u sa / (2 sqrt(disc)); four times their effect on r = (mid +- root)/den,
// plus 1e-6 (1 + |r|)); the full range when |den| < 1e-5 or the roots
// are not real; false when empty.
__device__ inline bool axis_range(float ca, float cu, float sa, float& lo, float& hi) {
    const float den = ca * ca - sa * sa;
    const float disc = ca * ca + cu * cu - sa * sa;  // discriminant of f / (4 sa^2)
    float a = -1.0f, b = 1.0f;
    if (disc > 0.0f && fabsf(den) > 1e-5f) {
        const float sq = sqrtf(disc);
        const float root = sa * sq, mid = ca * cu;
        const float r1 = (mid - root) / den, r2 = (mid + root) / den;
        const float ad = fabsf(den), w2 = ca * ca + sa * sa;
        const float e0 = (8.0f * kUlp * (fabsf(mid) + root) + 20.0f * kUlp * sa / sq) / ad;
        const float m1 = e0 + 12.0f * kUlp * fabsf(r1) * w2 / ad + 1e-6f * (1.0f + fabsf(r1));
        const float m2 = e0 + 12.0f * kUlp * fabsf(r2) * w2 / ad + 1e-6f * (1.0f + fabsf(r2));
        if (den > 0.0f) {  // f <= 0 between the roots r1 <= r2
            a = fmaxf(r1 - m1, -1.0f);
            b = fminf(r2 + m2, 1.0f);
            if (a > b) return false;
        } else {  // f <= 0 outside (r2, r1)
            const float hi2 = r2 + m2, lo1 = r1 - m1;
            const bool left = hi2 >= -1.0f, right = lo1 <= 1.0f;
            if (!left && !right) return false;
            if (!right) b = fminf(hi2, 1.0f);
            if (!left) a = fmaxf(lo1, -1.0f);
        }
    }
    lo = a;
    hi = b;
    return true;
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
    if (!axis_range(cax, cu, sa, ulo, uhi) || !axis_range(cax, cv, sa, vlo, vhi)) return false;
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
    float sa, ca;
    sincosf(alpha, &sa, &ca);
    return face_cells_sc(c, sa, ca, face, M, iu0, iu1, iv0, iv1);
}

// Work item of workgroup b of nb: the hardware deals workgroups to the 8
// XCDs in turn, so this gives each XCD one contiguous range of items (the
// neighbouring tiles of a view share candidates in that XCD's L2).  The
// batched kernels use it.
__device__ inline int64_t xcd_remap(int64_t b, int64_t nb) {
    int64_t x = b & 7, loc = b >> 3, q = nb >> 3, r = nb & 7;
    return x * q + (x < r ? x : r) + loc;
}

// Pixel rows per band of band_remap.
constexpr int kBandPx = 64;

// Work item of workgroup b of nb for a single view's kernels: items go in
// bands of g consecutive items (whole rows of tiles, kBandPx pixels high),
// band k to XCD k mod 8, so that each XCD keeps neighbouring tiles together
// in its L2 while the heavy regions of a picture (dense scene areas, the
// poles of a 360-degree map) spread over all XCDs instead of loading the few
// that one contiguous range per XCD would give them.  At 1920x1080 this took
// k_bin from 72 to 70 us and k_raster from 43 to 41 us for 1.4x and 1.1x
// their L2 fetches; grid order (no bands) was as fast but fetched 2.6x and
// 1.6x, 16-pixel bands 2.8x and 1.4x.  Items past the last whole round of 8
// bands map to themselves.
__device__ inline int64_t band_remap(int64_t b, int64_t nb, int64_t g) {
    const int64_t full = nb - nb % (8 * g);
    if (b >= full) return b;
    const int64_t x = b & 7, loc = b >> 3;
    return ((loc / g) * 8 + x) * g + loc % g;
}

__device__ inline float4 empty_cap0() { return make_float4(0.f, 0.f, 1.f, 0.f); }
__device__ inline float4 empty_cap1() { return make_float4(1.f, 0.f, kCapEmpty, 0.f); }

// Cosine of a binning cap's half radius from its sine.  The hardware square
// root (about 1 ulp) is ample: the cap tests carry a relative margin of 1e-6.
__device__ inline float bin_cos_half(float4 a) { return __builtin_amdgcn_sqrtf(fmaxf(0.0f, 1.0f - a.w * a.w)); }

// May a triangle (binning record a, ch_t = bin_cos_half(a), unit edge
// normals) cover a pixel of the tile with cap (c0, c1)?  Never false for a
// pair the rasterizer's FP32 test could cover.
// Written without branches (every lane evaluates every test and the
// results combine bitwise): in the binners' candidate loops, whose lanes
// hold different triangles, the short-circuit form's exec-mask branches
// cost 13% of the 16x16 block binner's time.
__device__ inline bool sub_may_see(float4 c0, float4 c1, float4 a, float ch_t, float3 n0, float3 n1, float3 n2) {
    const float dx = c0.x - a.x, dy = c0.y - a.y, dz = c0.z - a.z;
    const float chord2 = dx * dx + dy * dy + dz * dz;
    const float sm = c0.w * ch_t + c1.x * a.w;  // sin((rho_tile + rho_tri)/2)
    // caps apart (not for a useless triangle cap)
    const bool apart = (a.w < kBinWide) & (chord2 > 4.0f * sm * sm * (1.0f + 1e-6f) + 1e-12f);
    const float3 c = f3(c0.x, c0.y, c0.z);
    const float lim = -c1.y - 1e-6f;
    // the tile cap wholly outside one edge plane
    const float d0 = dot3(n0, c), d1 = dot3(n1, c), d2 = dot3(n2, c);
    const bool outside = (d0 < lim) | (d1 < lim) | (d2 < lim);
    return (c1.z != kCapEmpty) & ((c1.z == kCapWide) | !(apart | outside));
}

// sub_may_see with early returns (the same decision): in the rasterizers'
// cull, which tests each entry against one or two tiles only, skipping the
// plane tests of lanes whose caps are apart is 4% faster.
__device__ inline bool sub_may_see_lazy(float4 c0, float4 c1, float4 a, float ch_t, float3 n0, float3 n1,
                                        float3 n2) {
    if (c1.z == kCapEmpty) return false;
    if (c1.z == kCapWide) return true;
    if (a.w < kBinWide) {
        const float dx = c0.x - a.x, dy = c0.y - a.y, dz = c0.z - a.z;
        const float chord2 = dx * dx + dy * dy + dz * dz;
        const float sm = c0.w * ch_t + c1.x * a.w;
        if (chord2 > 4.0f * sm * sm * (1.0f + 1e-6f) + 1e-12f) return false;
    }
    const float3 c = f3(c0.x, c0.y, c0.z);
    const float lim = -c1.y - 1e-6f;
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
constexpr int kGatherPer = 4;                    // candidates per thread per gather block
constexpr int kGatherBlock = 256 * kGatherPer;   // one block's candidates; also the survivor list size

struct SuperShared {
    float4 cap[kSupTiles][2];
    float4 sup[2];
    int rect[64][4];
    uint32_t ppre[65];
    uint32_t spre[64][kSlices + 1];
    uint32_t rb[256], pre[256], wsum[4];
    uint32_t cnt[kSupTiles];
    uint32_t flag[kSupTiles];
    uint32_t npass;
    uint32_t fc[kSlices * 64];  // per-slice (level, face) triangle counts
    alignas(16) uint32_t bk[kSupTiles][kDepthBuckets];  // rows read and written as uint4
    alignas(16) uint16_t mark[kGatherBlock];            // row starts (row + 1) in one window of candidates
    uint32_t carry;                                     // row holding the window's first candidate
};
static_assert(offsetof(SuperShared, bk) % 16 == 0 && offsetof(SuperShared, mark) % 16 == 0,
              "rows read and written as uint4 are 16-byte aligned");
static_assert(kGatherPer == 4 && kGatherBlock == 4 * 256, "a thread reads its window marks as one uint2");
static_assert(kSupTiles * kDepthBuckets >= kGatherBlock, "survivor list fits in the bucket counters");

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

// Cell rectangles of every (level, face) for the gathering cap sh.sup, and
// the per-slice face counts.  All threads of the block call it after sh.sup
// is set (and visible).  Angles are never formed: caps carry sin and cos of
// their half radius, and radii add through the angle-sum identities.
__device__ inline void setup_rects(SuperShared& sh) {
    const int tid = threadIdx.x;
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


// Loads the four tile caps and the super-tile cap (rotated to the world
// frame) and the per-slice face counts, then the cell rectangles.  All
// threads of the block call it.
__device__ inline void super_setup(SuperShared& sh, const float4* caps, const float4* sups, const Rot& R,
                                   const uint32_t* face_count, bool present, int64_t tile, int64_t sidx) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    if (lane == 0) {
        float4 c0 = empty_cap0(), c1 = empty_cap1();
        if (present) load_tile_cap(caps, tile, R, c0, c1);
        sh.cap[w][0] = c0;
        sh.cap[w][1] = c1;
    }
    if (tid == 64) {
        float4 s0, s1;
        load_tile_cap(sups, sidx, R, s0, s1);
        sh.sup[0] = s0;
        sh.sup[1] = s1;
    }
    for (int q = tid; q < kSlices * 64; q += 256) sh.fc[q] = face_count[q];
    if (tid < kSupTiles) {
        sh.cnt[tid] = 0;
        sh.flag[tid] = 0;
    }
    __syncthreads();
    setup_rects(sh);
}

// Binning record of survivor `p` (cell-ordered position) for thread-level
// tests: visit(valid, a, bin_cos_half(a), n0, n1, n2, rank).
template <typename Visit>
__device__ inline void visit_record(const SceneView& S, bool valid, uint32_t p, Visit&& visit) {
    float4 a4 = make_float4(0.f, 0.f, 0.f, 0.f), b4 = a4, c4 = a4, d4 = a4;
    if (valid) {
        a4 = S.bincap[p];
        b4 = S.binnrm[3 * int64_t(p)];
        c4 = S.binnrm[3 * int64_t(p) + 1];
        d4 = S.binnrm[3 * int64_t(p) + 2];
    }
    visit(valid, a4, bin_cos_half(a4), f3(b4.x, b4.y, b4.z), f3(c4.x, c4.y, c4.z), f3(d4.x, d4.y, d4.z),
          __float_as_uint(b4.w));
}

// Streams the candidates of depth slices [s0, s1) through the test against
// the gathering cap sh.sup.  The rows of every (level, face, slice) are
// flattened into one list so that their cell ranges load and scan in one
// pass; each window of kGatherBlock candidates finds its rows from marks at
// the row starts and a block max-scan.  visit_chunk(list, n) is called by every thread for each chunk of
// at most 256 survivors (cell-ordered positions list[0..n)); it tests the
// caller's tiles and appends.  chunk_end() runs after each such call, by all
// threads (a point where the caller may synchronise).  All threads of the
// block call this with the same arguments.
template <typename VisitChunk, typename ChunkEnd>
__device__ inline void gather_slices(SuperShared& sh, const SceneView& S, int s0, int s1, VisitChunk&& visit_chunk,
                                     ChunkEnd&& chunk_end) {
    const int tid = threadIdx.x;
    const float4 sup0 = sh.sup[0], sup1 = sh.sup[1];
    const float3 cs = f3(sup0.x, sup0.y, sup0.z);
    const float sh_s = sup1.x, ch_s = sup1.y;
    const bool wide = sup1.w != 0.0f;
    reinterpret_cast<uint2*>(sh.mark)[tid] = make_uint2(0u, 0u);
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
    const uint32_t nrows_all = sh.ppre[64];
    uint32_t* const pass_list = &sh.bk[0][0];  // free while gathering
    const int lane = tid & 63, w = tid >> 6;
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
        if (tid == 0) sh.npass = 0;
        __syncthreads();
        for (uint32_t k0 = 0; k0 < total; k0 += kGatherBlock) {
            // stage 1: the super-tile cap test on up to kGatherPer candidates
            // per thread, their loads all in flight together; survivors are
            // compacted into pass_list
            // Thread t takes candidates k0 + 4t .. k0 + 4t + 3.  Their rows:
            // the row holding k0, and a mark (row + 1) where each later
            // non-empty row of the window starts; a running maximum over
            // the marks gives every candidate its row.
            if (uint32_t(tid) < nb && len > 0) {
                if (pre <= k0 && k0 - pre < len)
                    sh.carry = uint32_t(tid);
                else if (pre > k0 && pre - k0 < uint32_t(kGatherBlock))
                    sh.mark[pre - k0] = uint16_t(tid + 1);
            }
            __syncthreads();
            const uint2 m2 = reinterpret_cast<const uint2*>(sh.mark)[tid];
            reinterpret_cast<uint2*>(sh.mark)[tid] = make_uint2(0u, 0u);  // only this thread reads them
            uint32_t mk[kGatherPer] = {m2.x & 0xFFFFu, m2.x >> 16, m2.y & 0xFFFFu, m2.y >> 16};
#pragma unroll
            for (int u = 1; u < kGatherPer; ++u) mk[u] = max(mk[u], mk[u - 1]);
            uint32_t x = mk[kGatherPer - 1];
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const uint32_t y = __shfl_up(x, o, 64);
                if (lane >= o) x = max(x, y);
            }
            if (lane == 63) sh.wsum[w] = x;
            __syncthreads();
            uint32_t before = __shfl_up(x, 1, 64);
            if (lane == 0) before = 0u;
            for (int q = 0; q < w; ++q) before = max(before, sh.wsum[q]);
            before = max(before, sh.carry + 1u);
            uint32_t pos[kGatherPer];
            float4 a[kGatherPer];
#pragma unroll
            for (int u = 0; u < kGatherPer; ++u) {
                const uint32_t k = k0 + uint32_t(kGatherPer * tid + u);
                pos[u] = 0xFFFFFFFFu;
                if (k < total) {
                    const uint32_t row = max(before, mk[u]) - 1u;
                    pos[u] = sh.rb[row] + (k - sh.pre[row]);
                }
            }
#pragma unroll
            for (int u = 0; u < kGatherPer; ++u)
                a[u] = (pos[u] != 0xFFFFFFFFu) ? S.bincap[pos[u]] : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
            for (int u = 0; u < kGatherPer; ++u) {
                // evaluated by every lane, combined bitwise (no branches)
                const float dx = cs.x - a[u].x, dy = cs.y - a[u].y, dz = cs.z - a[u].z;
                const float chord2 = dx * dx + dy * dy + dz * dz;
                const float sm = sh_s * bin_cos_half(a[u]) + ch_s * a[u].w;
                const bool near = chord2 <= 4.0f * sm * sm * (1.0f + 1e-6f) + 1e-12f;
                const bool pass = (pos[u] != 0xFFFFFFFFu) & (wide | !(a[u].w < kBinWide) | near);
                if (pass) pass_list[atomicAdd(&sh.npass, 1u)] = pos[u];
            }
            __syncthreads();
            const uint32_t npass = sh.npass;
            __syncthreads();
            if (tid == 0) sh.npass = 0;  // next block's count; ordered by the syncs below
            // stage 2: the caller's tile tests on the survivors
            for (uint32_t c0 = 0; c0 < npass; c0 += 256) {
                visit_chunk(pass_list + c0, min(256u, npass - c0));
                chunk_end();
            }
            __syncthreads();
        }
        __syncthreads();
    }
}

// Counting sort of one wave's list (ranks) by depth bucket into `out`.
__device__ inline void bucket_sort_wave(const uint32_t* in, uint32_t cnt_any, uint32_t* bk, int shift, uint32_t* out) {
    const int lane = threadIdx.x & 63;
    const uint32_t cnt = __builtin_amdgcn_readfirstlane(cnt_any);  // wave-uniform: scalar loop control
    if (cnt < 2u) {
        if (cnt == 1u && lane == 0) out[0] = in[0];
        return;
    }
    reinterpret_cast<uint4*>(bk)[lane] = make_uint4(0u, 0u, 0u, 0u);  // 16-byte aligned rows of 256
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    for (uint32_t i0 = 0; i0 < cnt; i0 += 64) {
        const uint32_t i = i0 + uint32_t(lane);
        if (i < cnt) atomicAdd(&bk[in[i] >> shift], 1u);
    }
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
    for (uint32_t i0 = 0; i0 < cnt; i0 += 64) {
        const uint32_t i = i0 + uint32_t(lane);
        if (i < cnt) {
            const uint32_t r = in[i];
            out[atomicAdd(&bk[r >> shift], 1u)] = r;
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

}  // namespace vsr
