// Internal layouts and device helpers of libvsr (gfx950).
//
// Build flags matter for this file: everything is compiled with
// -ffp-contract=off so that a*b - c*d is two rounded products and one
// rounded difference.  That makes the edge-plane normal of a shared edge
// exactly the negation of its neighbour's (watertight coverage); fused
// multiply-adds are written explicitly with fmaf() where wanted.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/vsr.h"

namespace vsr {

constexpr int kTile = VSR_TILE;              // tile edge in pixels
constexpr int kTilePix = kTile * kTile;      // 64 = one wavefront
constexpr int kLevels = 9;                   // cube-map index levels 0..8
constexpr int kMaxLevel = kLevels - 1;
constexpr float kPi = 3.14159265358979323846f;
constexpr float kQuarterPi = 0.785398163397448310f;
constexpr float kHalfPi = 1.57079632679489662f;
constexpr uint32_t kNoHit = VSR_NO_HIT;
// Buffers reach the kernels through argument structs, job tables or void*,
// so the compiler sees generic pointers and emits flat loads and stores.  A
// flat operation also counts as an LDS operation: every wait for LDS data
// would then wait for outstanding global loads too (a prefetch would stall
// the next LDS read).  All buffers of the library are global device memory;
// this cast says so.
template <typename T>
__device__ inline T* to_global(T* p) {
    return (T*)(__attribute__((address_space(1))) T*)(uintptr_t)p;
}

// Initial z-buffer key: depth +inf in the high word, id NO_HIT in the low word.
constexpr uint64_t kKeyEmpty = (uint64_t(0x7F800000u) << 32) | uint64_t(kNoHit);

// Cap margins (radians).  The FP32 coverage test can differ from the exact
// spherical triangle by ~1e-7 rad; caps are widened far beyond that so that
// binning never rejects a (tile, triangle) pair the rasterizer would cover.
constexpr float kCapAbsMargin = 2e-5f;
constexpr float kCapRelMargin = 1e-6f;

__host__ __device__ constexpr int64_t align256(int64_t x) { return (x + 255) & ~int64_t(255); }

// Cells of level L: 6 faces of M x M, M = 2^L.  Cells of all levels are
// numbered consecutively; cell kNumBuckets marks culled triangles.
__host__ __device__ constexpr int64_t level_base(int L) { return 6 * (((int64_t(1) << (2 * L)) - 1) / 3); }
constexpr int64_t kNumBuckets = level_base(kLevels);

// Depth slices of the nearest-first order: slice s holds ranks
// [slice_begin(s), slice_begin(s+1)) with boundaries at n/64, n/16, n/4.
// The cap index is built per slice: index key = s * kNumBuckets + cell,
// culled triangles get kIndexKeys.
constexpr int kSlices = 4;
constexpr int64_t kIndexKeys = int64_t(kSlices) * kNumBuckets;
__host__ __device__ inline int64_t slice_begin(int64_t n, int s) {
    if (s <= 0) return 0;
    if (s >= kSlices) return n;
    return n >> (2 * (kSlices - s));
}
__host__ __device__ inline int slice_of(int64_t n, int64_t rank) {
    int s = 0;
    while (s + 1 < kSlices && slice_begin(n, s + 1) <= rank) ++s;
    return s;
}

// --------------------------------------------------------------- map ----
struct MapLayout {
    int32_t ntx, nty;
    int64_t ntiles;
    int64_t nsup;         // 16x16 super-tiles (2x2 tiles), row-major over ((ntx+1)/2) x ((nty+1)/2)
    int64_t nblk;         // 32x32 blocks (4x4 tiles), row-major over ((ntx+3)/4) x ((nty+3)/4)
    int64_t plane_bytes;  // all pixel data
    int64_t caps_off;     // float4 x 2 per tile
    int64_t sups_off;     // float4 x 2 per super-tile
    int64_t blks_off;     // float4 x 2 per block
    int64_t bytes;
};

__host__ __device__ inline MapLayout map_layout(int32_t w, int32_t h, int32_t fmt) {
    MapLayout m;
    m.ntx = (w + kTile - 1) / kTile;
    m.nty = (h + kTile - 1) / kTile;
    m.ntiles = int64_t(m.ntx) * m.nty;
    m.nsup = int64_t((m.ntx + 1) / 2) * ((m.nty + 1) / 2);
    m.plane_bytes = m.ntiles * kTilePix * (fmt == VSR_MAP_OCT16 ? 4 : 12);
    m.caps_off = align256(m.plane_bytes);
    m.nblk = int64_t((m.ntx + 3) / 4) * ((m.nty + 3) / 4);
    m.sups_off = m.caps_off + align256(m.ntiles * 32);
    m.blks_off = m.sups_off + align256(m.nsup * 32);
    m.bytes = m.blks_off + align256(m.nblk * 32);
    return m;
}

// Map with anti-aliasing data (built with VSR_MAP_AA): the plain layout,
// then one float per pixel, tile-major like the directions, holding the
// section 1.1.1 global delta (0 for a pixel without direction).
__host__ __device__ inline int64_t aa_delta_off(int32_t w, int32_t h, int32_t fmt) { return map_layout(w, h, fmt).bytes; }
__host__ __device__ inline int64_t aa_map_bytes(int32_t w, int32_t h, int32_t fmt) {
    MapLayout m = map_layout(w, h, fmt);
    return m.bytes + align256(m.ntiles * kTilePix * 4);
}

// Per-view constants of the map generator, computed on the host in double
// precision and rounded once to float.
struct MapParams {
    int32_t W, H, aov, fmt;
    int32_t ntx, nty;
    int32_t kind;       // +1: k > 0, 0: k == 0, -1: k < 0
    int32_t xmul;       // x = (2i+1-W) * xmul / xden, y = (2j+1-H) * xmul / yden
    float xden, yden;   // denominators (rounded) ...
    float xden_lo, yden_lo;  // ... and their rounding residuals
    float rxden, ryden;      // 1 / the exact denominators, rounded
    float k;            // projection type k (divisor of the arc functions)
    float half;         // Omega / 2 in radians
    float kt;           // tan(k*Omega/2) (k>0) or sin(k*Omega/2) (k<0)
    float kt_lo;        // rounding residual of kt
    float sig0;         // limit of sin(theta)/R at R = 0
    float l;            // cylindricity
    float c;            // anamorphic divisor l*(1-s)+s
    float rc;           // 1 / (l*(1-s)+s), rounded
    float rot[9];
    int32_t lens;       // map generator, VSR_LENS_*
    int32_t lens_n;     // screen array: number of screens
    int32_t distort;    // Universal: Brown-Conrady coefficients not all zero
    float fringe;       // AA maps: caps widened by asin(fringe / delta) (1/2: triangles, 5/4: lines)
    float lp[8];        // generator constants (set by the host, see make_map_params)
};

// ------------------------------------------------------------- setup ----
struct SetupLayout {
    int64_t n;
    int64_t nblocks;    // radix-sort blocks
    int64_t rec_off, cap_off, rcap_off, cell_list_off, cell_start_off, order_off, bincap_off, binnrm_off,
        face_count_off;
    int64_t rec_id_off, cap_id_off, key_a_off, val_a_off, key_b_off, val_b_off, bucket_off, hist_off;
    int64_t bytes;
};

constexpr int kSortThreads = 256;
constexpr int kSortItems = 8;
constexpr int kSortBlock = kSortThreads * kSortItems;  // 2048 keys per block

__host__ __device__ inline SetupLayout setup_layout(int64_t n) {
    SetupLayout s;
    s.n = n;
    s.nblocks = (n + kSortBlock - 1) / kSortBlock;
    int64_t o = 256;
    s.rec_off = o;        o += align256(n * 64);
    s.cap_off = o;        o += align256(n * 32);
    s.rcap_off = o;       o += align256(n * 16);
    s.cell_list_off = o;  o += align256(n * 4);
    s.cell_start_off = o; o += align256((kIndexKeys + 1) * 4);
    s.face_count_off = o; o += align256(int64_t(kSlices) * 64 * 4);
    s.order_off = o;      o += align256(n * 4);
    s.bincap_off = o;     o += align256(n * 16);
    s.binnrm_off = o;     o += align256(n * 48);
    s.rec_id_off = o;     o += align256(n * 64);
    s.cap_id_off = o;     o += align256(n * 32);
    s.key_a_off = o;      o += align256(n * 4);
    s.val_a_off = o;      o += align256(n * 4);
    s.key_b_off = o;      o += align256(n * 4);
    s.val_b_off = o;      o += align256(n * 4);
    s.bucket_off = o;     o += align256(n * 4);
    s.hist_off = o;       o += align256((256 * (s.nblocks > 0 ? s.nblocks : 1) + 256) * 4);
    s.bytes = o;
    return s;
}

// Depth buckets of the nearest-first order: bucket of rank r is r >> shift.
constexpr int kDepthBuckets = 256;
__host__ __device__ inline int bucket_shift(int64_t n) {
    int s = 0;
    while ((int64_t(kDepthBuckets) << s) < n) ++s;
    return s;
}

// --------------------------------------------------------------- bins ---
struct BinLayout {
    int64_t ntiles;
    int64_t counts_off;
    int64_t lists_off;
    int64_t bytes;
};

__host__ __device__ inline BinLayout bin_layout(int32_t w, int32_t h, int32_t depth) {
    MapLayout m = map_layout(w, h, VSR_MAP_F32);
    BinLayout b;
    b.ntiles = m.ntiles;
    b.counts_off = 256;  // first 256 bytes: status words (overflowed tile count)
    b.lists_off = b.counts_off + align256(m.ntiles * 4);
    b.bytes = b.lists_off + align256(m.ntiles * int64_t(depth) * 4);
    return b;
}

// ------------------------------------------------------ device helpers --
__device__ inline float3 f3(float x, float y, float z) { return make_float3(x, y, z); }
__device__ inline float3 sub3(float3 a, float3 b) { return f3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ inline float3 add3(float3 a, float3 b) { return f3(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ inline float3 scale3(float3 a, float s) { return f3(a.x * s, a.y * s, a.z * s); }
__device__ inline float dot3(float3 a, float3 b) { return fmaf(a.z, b.z, fmaf(a.y, b.y, a.x * b.x)); }
// Nearest-first order: triangles are sorted by the top kDepthKeyBits bits
// of their (non-negative) depth lower bound, whose bits order like the
// values.  Ranks with equal keys keep id order, so a bound valid for a rank
// and every later rank is the first rank's lower bound with the dropped low
// bits cleared (depth_key_floor), not its lower bound itself.
constexpr int kDepthKeyBits = 24;
__device__ inline uint32_t depth_key(float lb) { return __float_as_uint(lb) >> (32 - kDepthKeyBits); }
__device__ inline float depth_key_floor(float lb) {
    return __uint_as_float(__float_as_uint(lb) & ~((1u << (32 - kDepthKeyBits)) - 1u));
}

// Unit roundoff of FP32, 2^-24: the bound on the relative error of one
// rounded operation, in the error budgets of conservative tests.
constexpr float kUlp = 5.9604645e-8f;

// Cross product with separately rounded products (no contraction).
__device__ inline float3 cross3(float3 a, float3 b) {
    return f3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}

// Wave-wide reductions (64 lanes).
__device__ inline float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ inline float wave_max(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ inline uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        uint32_t w = __shfl_xor(v, o, 64);
        v = w > v ? w : v;
    }
    return v;
}

// Wave-wide maximum of unsigned values with DPP row shifts and row
// broadcasts; lanes that a DPP step does not feed read 0 (the identity).
// Lane 63 ends with the maximum, returned to every lane as a scalar.
template <int kCtrl, int kRowMask, bool kBound>
__device__ inline uint32_t dpp_max_step(uint32_t v) {
    return max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, kCtrl, kRowMask, 0xF, kBound));
}
__device__ inline uint32_t wave_max_u32_dpp(uint32_t v) {
    v = dpp_max_step<0x111, 0xF, true>(v);   // row_shr:1
    v = dpp_max_step<0x112, 0xF, true>(v);   // row_shr:2
    v = dpp_max_step<0x114, 0xF, true>(v);   // row_shr:4
    v = dpp_max_step<0x118, 0xF, true>(v);   // row_shr:8
    v = dpp_max_step<0x142, 0xA, false>(v);  // row_bcast:15 into rows 1 and 3
    v = dpp_max_step<0x143, 0xC, false>(v);  // row_bcast:31 into rows 2 and 3
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

// Octahedral unit-vector encoding (two fp16).  The all-ones word marks a
// pixel without a direction.
constexpr uint32_t kOctInvalid = 0xFFFFFFFFu;

__device__ inline uint32_t oct_encode(float3 g) {
    float s = fabsf(g.x) + fabsf(g.y) + fabsf(g.z);
    if (!(s > 0.0f)) return kOctInvalid;
    float x = g.x / s, y = g.y / s;
    if (g.z < 0.0f) {
        float ox = (1.0f - fabsf(y)) * (x >= 0.0f ? 1.0f : -1.0f);
        float oy = (1.0f - fabsf(x)) * (y >= 0.0f ? 1.0f : -1.0f);
        x = ox;
        y = oy;
    }
    _Float16 hx = (_Float16)x, hy = (_Float16)y;
    uint16_t bx, by;
    __builtin_memcpy(&bx, &hx, 2);
    __builtin_memcpy(&by, &hy, 2);
    return uint32_t(bx) | (uint32_t(by) << 16);
}

__device__ inline float3 oct_decode(uint32_t w) {
    if (w == kOctInvalid) return f3(0.0f, 0.0f, 0.0f);
    uint16_t bx = uint16_t(w & 0xFFFFu), by = uint16_t(w >> 16);
    _Float16 hx, hy;
    __builtin_memcpy(&hx, &bx, 2);
    __builtin_memcpy(&hy, &by, 2);
    float x = (float)hx, y = (float)hy;
    float z = 1.0f - fabsf(x) - fabsf(y);
    if (z < 0.0f) {
        float ox = (1.0f - fabsf(y)) * (x >= 0.0f ? 1.0f : -1.0f);
        float oy = (1.0f - fabsf(x)) * (y >= 0.0f ? 1.0f : -1.0f);
        x = ox;
        y = oy;
    }
    float inv = 1.0f / sqrtf(fmaf(x, x, fmaf(y, y, z * z)));
    return f3(x * inv, y * inv, z * inv);
}

// Tile caps of a map buffer (2 x float4 per tile, after the pixel planes).
__host__ __device__ inline const float4* map_caps(const void* map, int64_t ntiles, int32_t fmt) {
    return reinterpret_cast<const float4*>(reinterpret_cast<const char*>(map) +
                                           align256(ntiles * kTilePix * (fmt == VSR_MAP_OCT16 ? 4 : 12)));
}

// Super-tile caps of a map buffer (2 x float4 per 16x16 super-tile, after
// the tile caps).
__host__ __device__ inline const float4* map_sups(const void* map, int64_t ntiles, int32_t fmt) {
    return reinterpret_cast<const float4*>(reinterpret_cast<const char*>(map_caps(map, ntiles, fmt)) +
                                           align256(ntiles * 32));
}

// Block caps of a map buffer (2 x float4 per 32x32 block, after the
// super-tile caps).
__host__ __device__ inline const float4* map_blks(const void* map, int64_t ntiles, int32_t fmt, int32_t ntx,
                                                  int32_t nty) {
    const int64_t nsup = int64_t((ntx + 1) / 2) * ((nty + 1) / 2);
    return reinterpret_cast<const float4*>(reinterpret_cast<const char*>(map_sups(map, ntiles, fmt)) +
                                           align256(nsup * 32));
}

// Camera -> world rotation of a view (row-major), applied to the camera-frame
// map: the map depends only on the lens (size, AOV, k, l, s, Omega), so one
// map serves every orientation.
struct Rot {
    float m[9];
};

__host__ __device__ inline Rot rot_of(const float* r) {
    Rot R;
    for (int q = 0; q < 9; ++q) R.m[q] = r[q];
    return R;
}

// World direction of a camera-frame direction (fixed FP32 operation order).
__device__ inline float3 rotate_dir(const Rot& R, float3 v) {
    return f3(fmaf(R.m[2], v.z, fmaf(R.m[1], v.y, R.m[0] * v.x)),
              fmaf(R.m[5], v.z, fmaf(R.m[4], v.y, R.m[3] * v.x)),
              fmaf(R.m[8], v.z, fmaf(R.m[7], v.y, R.m[6] * v.x)));
}

// Load the camera-frame direction of pixel `lane` of tile `tile`.
__device__ inline float3 load_dir_cam(const void* map, int32_t fmt, int64_t ntiles, int64_t tile, int lane) {
    if (fmt == VSR_MAP_OCT16) {
        const uint32_t* p = reinterpret_cast<const uint32_t*>(map);
        return oct_decode(p[tile * kTilePix + lane]);
    }
    const float* p = reinterpret_cast<const float*>(map);
    int64_t plane = ntiles * kTilePix;
    int64_t q = tile * kTilePix + lane;
    return f3(p[q], p[plane + q], p[2 * plane + q]);
}

// World direction of pixel `lane` of tile `tile` (zero: no direction).
__device__ inline float3 load_dir(const void* map, int32_t fmt, int64_t ntiles, int64_t tile, int lane,
                                  const Rot& R) {
    return rotate_dir(R, load_dir_cam(map, fmt, ntiles, tile, lane));
}

// World-frame cap of tile `tile`: the camera-frame centre rotated.  The
// rotation's FP32 rounding (a few 1e-7 rad) is far inside the cap margin
// (2e-5 rad), so the cap still bounds every rotated pixel direction.
__device__ inline void load_tile_cap(const float4* caps, int64_t tile, const Rot& R, float4& c0, float4& c1) {
    c0 = caps[2 * tile];
    c1 = caps[2 * tile + 1];
    const float3 c = rotate_dir(R, f3(c0.x, c0.y, c0.z));
    c0 = make_float4(c.x, c.y, c.z, c0.w);
}

// Tile of wave w (0..3) in super-tile sidx (2x2 tiles, row-major over
// ((ntx+1)/2) columns); false when outside the map.
__host__ __device__ inline bool super_tile_of(int64_t sidx, int w, int ntx, int nty, int64_t& tile, int& tx, int& ty) {
    const int nsx = (ntx + 1) / 2;
    const int sx = int(sidx % nsx), sy = int(sidx / nsx);
    tx = 2 * sx + (w & 1);
    ty = 2 * sy + (w >> 1);
    tile = int64_t(ty) * ntx + tx;
    return tx < ntx && ty < nty;
}

// Binning record of a triangle, stored in cell order (entry k belongs to
// cell_list[k]) so that a run of cells streams as coalesced 64-byte loads:
//   a = (cap centre xyz, sin(rho/2), or kBinWide for a useless cap)
//   b = (n0 xyz, rank bits), c = (n1 xyz, 0), d = (n2 xyz, 0)
// with n_i the oriented unit edge-plane normals.
constexpr float kBinWide = 2.0f;

// Tile cap record: c0 = (centre.xyz, sin(rho/2)), c1 = (cos(rho/2), sin(rho), flags, 0)
constexpr float kCapWide = 1.0f;   // cap radius >= pi/2: no culling possible
constexpr float kCapEmpty = 2.0f;  // no pixel with a direction
// Triangle cap record: same layout, widened by the FP32 margins; flags
// kCapWide when the cap is useless for culling.  Its fourth word c1.w holds
// the sine of half the exact (unwidened) radius of the section 1.1.2
// smallest circle, whose centre is c0.xyz also for wide caps; 0 when the
// circle is degenerate (no miter).

// Conservative test: may triangle (cap tc0/tc1, oriented unit edge normals
// n0..n2) cover any pixel of the tile (cap c0/c1)?  Never returns false for
// a pair the rasterizer's FP32 test could cover.
__device__ inline bool tile_may_see(float4 c0, float4 c1, float4 t0, float4 t1, float3 n0, float3 n1,
                                    float3 n2) {
    if (c1.z == kCapEmpty) return false;
    if (c1.z == kCapWide) return true;
    if (t1.z != kCapWide) {
        float dx = c0.x - t0.x, dy = c0.y - t0.y, dz = c0.z - t0.z;
        float chord2 = dx * dx + dy * dy + dz * dz;
        // sin((rho_tile + rho_tri)/2) by the angle-sum identity
        float s = c0.w * t1.x + c1.x * t0.w;
        if (chord2 > 4.0f * s * s * (1.0f + 1e-6f) + 1e-12f) return false;
    }
    float3 c = f3(c0.x, c0.y, c0.z);
    float lim = -c1.y - 1e-6f;
    if (dot3(n0, c) < lim || dot3(n1, c) < lim || dot3(n2, c) < lim) return false;
    return true;
}

// Cap of a 16x16 super-tile bounding its four tile caps, written as
//   sup0 = (centre, sin of half the radius), sup1 = (same sine, its cosine,
//   1 if any tile has a direction, 1 if the cap is wide (radius >= pi/2)).
// Angles are never formed: half radii add through the angle-sum identities
// on the half-chord between centres.  The margin (1e-6 relative, 1e-6
// absolute on the half-radius sine) also covers the rotation of the centres
// into the world frame, which is applied after this (the tile caps carry
// 2e-5 rad over their pixels, so pixels stay well inside).
__device__ inline void super_cap_of(const float4 (&cap)[4][2], float4& sup0, float4& sup1) {
    bool any0 = false, wide0 = false;
    float3 sum = f3(0.f, 0.f, 0.f);
    for (int q = 0; q < 4; ++q) {
        const float4 c0 = cap[q][0], c1 = cap[q][1];
        if (c1.z == kCapEmpty) continue;
        any0 = true;
        if (c1.z == kCapWide) wide0 = true;
        sum = add3(sum, f3(c0.x, c0.y, c0.z));
    }
    float3 c = f3(0.f, 0.f, 1.f);
    float sh_ = 1.0f, ch_ = 0.0f;
    if (any0 && !wide0) {
        const float len = sqrtf(dot3(sum, sum));
        if (len > 1e-3f) {
            c = scale3(sum, 1.0f / len);
            sh_ = 0.0f;
            ch_ = 1.0f;
            for (int q = 0; q < 4; ++q) {
                const float4 c0 = cap[q][0], c1 = cap[q][1];
                if (c1.z == kCapEmpty) continue;
                const float3 d = sub3(c, f3(c0.x, c0.y, c0.z));
                const float st = fminf(1.0f, 0.5f * sqrtf(dot3(d, d)));
                const float ct = sqrtf(fmaxf(0.0f, 1.0f - st * st));
                const float sq = st * c1.x + ct * c0.w, cq = ct * c1.x - st * c0.w;
                if (!(cq > 0.0f)) {
                    wide0 = true;
                } else if (sq > sh_) {
                    sh_ = sq;
                    ch_ = cq;
                }
            }
            sh_ = sh_ * (1.0f + 1e-6f) + 1e-6f;
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
    sup0 = make_float4(c.x, c.y, c.z, sh_);
    sup1 = make_float4(sh_, ch_, any0 ? 1.0f : 0.0f, wide0 ? 1.0f : 0.0f);
}

// A super-tile cap (sup0, sup1 as written by super_cap_of) in the tile-cap
// layout that super_cap_of reads for its children.
__device__ inline void sup_as_child(float4 sup0, float4 sup1, float4& c0, float4& c1) {
    c0 = sup0;
    const float flag = sup1.z == 0.0f ? kCapEmpty : (sup1.w != 0.0f ? kCapWide : 0.0f);
    c1 = make_float4(sup1.y, 2.0f * sup1.x * sup1.y, flag, 0.0f);
}

}  // namespace vsr
