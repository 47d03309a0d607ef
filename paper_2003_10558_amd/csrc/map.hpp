// Perspective vector map (Universal Perspective model, or one of the other
// generators of section 2.2) and per-tile caps.
//
// One wavefront per 8x8 tile, one lane per pixel.  Each lane turns its pixel
// centre into view coordinates (angle-of-view normalisation, section 2),
// applies the 2D->3D transform of section 2.1.2 in FP32 with the accurate
// device math library and stores the camera-frame direction tile-major (x, y
// and z planes, or one octahedral fp16 pair).  The wave then reduces the
// tile's bounding cap: the normalised mean direction and the largest chord
// to it, widened by a safety margin.
//
// Each 16x16 super-tile also gets a cap bounding its four tile caps, and
// each 32x32 block one bounding its four super-tile caps (used by the
// binner).
//
// The map depends only on the lens (size, angle of view, k, l, s, Omega): as
// in the paper, where the vector map is computed once and kept as a texture,
// one map serves every orientation.  Consumers rotate directions and cap
// centres into the world frame as they load them (load_dir, load_tile_cap).
#pragma once
#include "vsr_internal.h"

namespace vsr {

// Double-float helpers (value = hi + lo, |lo| <= ulp(hi)/2).
__device__ inline void two_sum(float a, float b, float& s, float& e) {
    s = a + b;
    float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// asin(q) for |q| <= 1 given q = qh + ql in double-float.  Near |q| = 1 asin
// is ill-conditioned (the rim of sine-type projections); there it is taken
// as pi/2 - 2 asin(sqrt((1-|q|)/2)) with 1-|q| formed exactly.
__device__ inline float asin_df(float qh, float ql) {
    float ah = fabsf(qh), al = qh < 0.0f ? -ql : ql;
    float a;
    if (ah <= 0.5f) {
        a = asinf(ah + al);
    } else {
        float t = (1.0f - ah) - al;  // 1 - ah is exact for ah in [0.5, 1]
        a = kHalfPi - 2.0f * asinf(sqrtf(fmaxf(0.0f, 0.5f * t)));
    }
    return qh < 0.0f ? -a : a;
}

// Section 2.3 Brown-Conrady distortion of view coordinates: radial
// (1 + k1 r^2 + k2 r^4), thin prism (p . f) f, decentering q r^2;
// c = (k1, k2, p1, p2, q1, q2).
__device__ inline void lens_distort(const float* c, float& x, float& y) {
    float r2 = fmaf(x, x, y * y);
    float radial = fmaf(r2, fmaf(c[1], r2, c[0]), 1.0f);
    float prism = fmaf(c[2], x, c[3] * y);
    float nx = fmaf(x, radial, fmaf(prism, x, c[4] * r2));
    float ny = fmaf(y, radial, fmaf(prism, y, c[5] * r2));
    x = nx;
    y = ny;
}

// Universal Perspective (section 2.1.2) camera direction of pixel (i, j);
// false when the pixel is outside the projection's domain.
__device__ inline bool universal_direction(const MapParams& P, int i, int j, float3& out) {
    float nx = float((2 * i + 1 - P.W) * P.xmul), ny = float((2 * j + 1 - P.H) * P.xmul);
    // the per-view divisions are products with rounded reciprocals and the
    // per-pixel ones hardware reciprocals (about 1 ulp each, far inside the
    // map's accuracy bound of 1e-6 rad; the double-float path below takes
    // the exact residuals of whatever x and y hold)
    float x = nx * P.rxden;
    float y = ny * P.ryden;
    if (P.distort) lens_distort(P.lp, x, y);
    float R = sqrtf(fmaf(x, x, P.l * (y * y)));
    float theta;
    if (P.kind > 0) {
        theta = atanf(P.kt * R) / P.k;
    } else if (P.kind < 0) {
        // sin(k Omega/2) R in double-float: x, y, R^2, R and the product
        // (the rounding residuals of x and y are known only undistorted)
        float xl = P.distort ? 0.0f : (fmaf(-x, P.xden, nx) - x * P.xden_lo) * P.rxden;
        float yl = P.distort ? 0.0f : (fmaf(-y, P.yden, ny) - y * P.yden_lo) * P.ryden;
        float xx = x * x, xxe = fmaf(x, x, -xx) + 2.0f * x * xl;
        float yy = y * y, yye = fmaf(y, y, -yy) + 2.0f * y * yl;
        float ly = P.l * yy, lye = fmaf(P.l, yy, -ly) + P.l * yye;
        float Xh, Xe;
        two_sum(xx, ly, Xh, Xe);
        Xe += xxe + lye;
        float Rh = sqrtf(Xh);
        float Rl = Rh > 0.0f ? (fmaf(-Rh, Rh, Xh) + Xe) * (0.5f * __builtin_amdgcn_rcpf(Rh)) : 0.0f;
        float qh = P.kt * Rh;
        float ql = fmaf(P.kt, Rh, -qh) + P.kt * Rl + P.kt_lo * Rh;
        float s, e;
        two_sum(qh, ql, s, e);
        if (fabsf(s) > 1.0f || (fabsf(s) == 1.0f && (s > 0.0f ? e > 0.0f : e < 0.0f))) return false;
        theta = asin_df(s, e) / P.k;
        R = Rh;
    } else {
        theta = P.half * R;
    }
    float sn, cs;
    sincosf(theta, &sn, &cs);
    float sig = R > 0.0f ? sn * __builtin_amdgcn_rcpf(R) : P.sig0;
    float v0 = x * sig, v1 = (y * sig) * P.rc, v2 = cs;
    float inv = __builtin_amdgcn_rsqf(fmaf(v0, v0, fmaf(v1, v1, v2 * v2)));
    out = f3(v0 * inv, v1 * inv, v2 * inv);
    return true;
}

__device__ inline float3 normalized(float x, float y, float z) {
    float inv = 1.0f / sqrtf(fmaf(x, x, fmaf(y, y, z * z)));
    return f3(x * inv, y * inv, z * inv);
}

// Picture segment of pixel (i, j): cube face, screen or eye (0 for the
// one-piece maps).  Texture coordinates are ratios of integers, so the
// segment index is exact integer arithmetic.
__device__ inline int pixel_segment(const MapParams& P, int i) {
    switch (P.lens) {
    case VSR_LENS_CUBE: return min(5, (3 * (2 * i + 1)) / P.W);
    case VSR_LENS_SCREENS: return min(P.lens_n - 1, (P.lens_n * (2 * i + 1)) / (2 * P.W));
    case VSR_LENS_VR: return 2 * i + 1 > P.W ? 1 : 0;
    default: return 0;
    }
}

// Camera direction of pixel (i, j) for the view's map generator (section
// 2.1.2, or the maps of section 2.2); false when the pixel has none.
__device__ inline bool pixel_direction(const MapParams& P, int i, int j, float3& out) {
    switch (P.lens) {
    case VSR_LENS_EQUIRECT: {  // section 2.2.4: longitude pi (2fs - 1), polar angle pi ft from -y
        float sl, cl, sp, cp;
        sincospif(float(2 * i + 1 - P.W) / float(P.W), &sl, &cl);
        sincospif(float(2 * j + 1) / float(2 * P.H), &sp, &cp);
        out = f3(sl * sp, -cp, cl * sp);
        return true;
    }
    case VSR_LENS_CUBE: {  // section 2.2.7: six 90-degree faces side by side
        const int face = pixel_segment(P, i);
        // face-local (fract(6 fs) - 1/2, ft - 1/2, 1/2), numerators exact
        float u = float(2 * (3 * (2 * i + 1) - P.W * face) - P.W) / float(2 * P.W);
        float v = float(2 * j + 1 - P.H) / float(2 * P.H);
        float3 d = normalized(u, v, 0.5f);
        switch (face) {  // rows of the face rotation; face 3 is the forward face
        case 0: out = f3(d.z, -d.x, -d.y); break;
        case 1: out = f3(-d.z, d.x, -d.y); break;
        case 2: out = f3(d.x, -d.y, -d.z); break;
        case 3: out = d; break;
        case 4: out = f3(d.x, d.z, -d.y); break;
        default: out = f3(-d.x, -d.z, -d.y); break;
        }
        return true;
    }
    case VSR_LENS_SCREENS: {  // section 2.2.8: n flat screens, screen s turned about y
        const int n = P.lens_n, s = pixel_segment(P, i);
        float u = float(n * (2 * i + 1) - 2 * P.W * s - P.W) / float(P.W);
        float v = float(n * (2 * j + 1 - P.H)) / float(P.W);
        float3 d = normalized(u, v, P.lp[0]);
        float sn, cs;
        sincosf(float(2 * s + 1 - n) * P.lp[1], &sn, &cs);
        out = f3(fmaf(cs, d.x, sn * d.z), d.y, fmaf(-sn, d.x, cs * d.z));
        return true;
    }
    case VSR_LENS_VR: {  // section 2.2.9: two eyes, IPD offset, radial lens distortion
        const int t = 2 * i + 1;
        const float eye = t > P.W ? 1.0f : (t < P.W ? -1.0f : 0.0f);
        float x = (float(2 * (t % P.W) - P.W) / float(P.W) + eye * P.lp[1]) * P.lp[5];
        float y = float(2 * j + 1 - P.H) / float(P.H);
        float R2 = fmaf(x, x, y * y);
        float f = fmaf(R2, fmaf(P.lp[3], R2, P.lp[2]), 1.0f) * P.lp[4];
        out = normalized(x * f, y * f, P.lp[0]);
        return true;
    }
    case VSR_LENS_DOME: {  // section 2.2.3: fisheye about the zenith +y, tilted about x
        // outside the inscribed circle: exact integer test of R^2 > 1
        const int64_t nx = 2 * i + 1 - P.W, ny = P.H - 2 * j - 1;
        if (nx * nx * int64_t(P.H) * P.H + ny * ny * int64_t(P.W) * P.W > int64_t(P.W) * P.W * int64_t(P.H) * P.H)
            return false;
        float x = float(nx) / float(P.W), y = float(ny) / float(P.H);
        float R = sqrtf(fmaf(x, x, y * y));
        float sn, cs;
        sincosf(R * P.lp[0], &sn, &cs);
        float sr = R > 0.0f ? sn / R : P.lp[0];
        float3 d = normalized(x * sr, cs, fmaf(y, sr, P.lp[3]));
        out = f3(d.x, fmaf(d.y, P.lp[2], d.z * P.lp[1]), fmaf(-d.y, P.lp[1], d.z * P.lp[2]));
        return true;
    }
    case VSR_LENS_PANORAMA: {  // section 2.2.2: unit cylinder, height from the aspect ratio
        float x = float(2 * i + 1 - P.W) * P.lp[0], y = float(2 * j + 1 - P.H) * P.lp[0];
        float sn, cs;
        sincosf(x, &sn, &cs);
        out = normalized(sn, y, cs);
        return true;
    }
    default:
        return universal_direction(P, i, j, out);
    }
}

// Derivative of the camera-frame map along one pixel axis at a pixel with
// direction g: central difference of the two neighbours gp (next) and gm
// (previous), one-sided where a neighbour is outside the picture, has no
// direction or lies in another segment of the picture (cube face, screen,
// eye: not adjacent on the sphere), zero when neither counts (okp, okm say
// which count).
__device__ inline float3 central_diff(float3 gp, bool okp, float3 gm, bool okm, float3 g) {
    if (okp && okm) return f3(0.5f * (gp.x - gm.x), 0.5f * (gp.y - gm.y), 0.5f * (gp.z - gm.z));
    if (okp) return sub3(gp, g);
    if (okm) return sub3(g, gm);
    return f3(0.f, 0.f, 0.f);
}

// Direction g and flag ok of lane `inner` when `use_inner`, else ge and oke
// of lane `ring` (all lanes of the wave call it together).
__device__ inline void neighbour(bool use_inner, int inner, int ring, float3 g, bool ok, float3 ge, bool oke,
                                 float3& gn, bool& okn) {
    const float3 a = f3(__shfl(g.x, inner, 64), __shfl(g.y, inner, 64), __shfl(g.z, inner, 64));
    const float3 b = f3(__shfl(ge.x, ring, 64), __shfl(ge.y, ring, 64), __shfl(ge.z, ring, 64));
    const int oa = __shfl(int(ok), inner, 64), ob = __shfl(int(oke), ring, 64);
    gn = use_inner ? a : b;
    okn = (use_inner ? oa : ob) != 0;
}

// Section 1.1.1 global delta of the lane's pixel (i, j) in 8x8 tile (tx, ty):
// the reciprocal of the largest component of fwidth(G) = |dG/di| + |dG/dj|
// (+inf when the map does not vary; 0 for a pixel without direction).  The
// four neighbours' directions inside the tile are those the neighbouring
// lanes hold (the same evaluation, so the same bits); the 32 pixels around
// the tile take one more evaluation by lanes 0..31 (right, left, lower,
// upper side, 8 each).  All lanes of the wave call it together.
__device__ inline float tile_pixel_delta(const MapParams& P, int tx, int ty, int i, int j, int lane, float3 g,
                                         bool ok) {
    const int x = lane & (kTile - 1), y = lane >> 3;
    float3 ge = f3(0.f, 0.f, 0.f);
    bool oke = false;
    if (lane < 4 * kTile) {
        const int side = lane >> 3, q = lane & (kTile - 1);
        const int ie = side == 0 ? tx * kTile + kTile : (side == 1 ? tx * kTile - 1 : tx * kTile + q);
        const int je = side < 2 ? ty * kTile + q : (side == 2 ? ty * kTile + kTile : ty * kTile - 1);
        if (ie >= 0 && ie < P.W && je >= 0 && je < P.H) oke = pixel_direction(P, ie, je, ge);
    }
    float3 gr, gl, gd, gu;
    bool okr, okl, okd, oku;
    neighbour(x < kTile - 1, (lane + 1) & 63, y, g, ok, ge, oke, gr, okr);
    neighbour(x > 0, (lane + 63) & 63, kTile + y, g, ok, ge, oke, gl, okl);
    neighbour(y < kTile - 1, (lane + kTile) & 63, 2 * kTile + x, g, ok, ge, oke, gd, okd);
    neighbour(y > 0, (lane + 64 - kTile) & 63, 3 * kTile + x, g, ok, ge, oke, gu, oku);
    if (!ok) return 0.0f;
    const int seg = pixel_segment(P, i);
    okr = okr && pixel_segment(P, i + 1) == seg;
    okl = okl && pixel_segment(P, i - 1) == seg;
    const float3 a = central_diff(gr, okr, gl, okl, g), b = central_diff(gd, okd, gu, oku, g);
    const float f = fmaxf(fabsf(a.x) + fabsf(b.x), fmaxf(fabsf(a.y) + fabsf(b.y), fabsf(a.z) + fabsf(b.z)));
    return f > 0.0f ? 1.0f / f : __int_as_float(0x7F800000);
}

// Widens a tile cap by the angle asin(f) of a fringe f (sine of the angle),
// times 1 + 1e-3, plus 1e-6 rad (a cap reaching pi/2 becomes wide).  No
// transcendental: asin(f) <= f / sqrt(1 - f^2), and with half radius a and
// half widening b, sin(a + b) <= sin(a) + cos(a) b.
__device__ inline void dilate_cap(float4& c0, float4& c1, float f) {
    if (c1.z == kCapEmpty || c1.z == kCapWide) return;
    float sh = 1.0f;
    if (f < 0.5f) {
        const float b = 0.5f * (f * __builtin_amdgcn_rsqf(1.0f - f * f) * (1.0f + 2e-3f) + 1e-6f);
        sh = fmaf(c1.x, b, c0.w) * (1.0f + 1e-7f);
    }
    if (!(sh < 0.70710678f)) {  // radius >= pi/2
        c0.w = 1.f;
        c1 = make_float4(0.f, 1.f, kCapWide, 0.f);
        return;
    }
    const float chh = sqrtf(1.0f - sh * sh);
    c0.w = sh;
    c1.x = chh;
    c1.y = 2.0f * sh * chh;
}

// Cap of the directions held by the lanes with ok=true (wave-uniform result).
__device__ inline void tile_cap(float3 g, bool ok, float4& c0, float4& c1) {
    uint64_t m = __ballot(ok);
    if (m == 0) {
        c0 = make_float4(0.f, 0.f, 1.f, 0.f);
        c1 = make_float4(1.f, 0.f, kCapEmpty, 0.f);
        return;
    }
    float sx = wave_sum(ok ? g.x : 0.f), sy = wave_sum(ok ? g.y : 0.f), sz = wave_sum(ok ? g.z : 0.f);
    float len = sqrtf(sx * sx + sy * sy + sz * sz);
    float n = (float)__popcll(m);
    if (!(len > 1e-3f * n)) {  // directions spread all round: no useful cap
        c0 = make_float4(0.f, 0.f, 1.f, 1.f);
        c1 = make_float4(0.f, 1.f, kCapWide, 0.f);
        return;
    }
    const float il = 1.0f / len;
    float3 c = f3(sx * il, sy * il, sz * il);
    float3 d = sub3(g, c);
    float ch2 = wave_max(ok ? d.x * d.x + d.y * d.y + d.z * d.z : 0.f);
    // Half radius a = asin(h), h = half the largest chord, widened by the
    // margins to a + delta, delta = a kCapRelMargin + kCapAbsMargin / 2.
    // No transcendental: asin(h) <= (pi/2) h bounds delta, and
    // sin(a + delta) <= h + cos(a) delta, so the cap is at least as wide as
    // the margins ask.
    const float h = fminf(1.0f, 0.5f * sqrtf(ch2));
    const float delta = kHalfPi * h * kCapRelMargin + 0.5f * kCapAbsMargin;
    const float sh = fmaf(sqrtf(fmaxf(0.0f, 1.0f - h * h)), delta, h) * (1.0f + 1e-7f);
    if (!(sh < 0.70710678f)) {  // radius >= pi/2
        c0 = make_float4(c.x, c.y, c.z, 1.f);
        c1 = make_float4(0.f, 1.f, kCapWide, 0.f);
        return;
    }
    const float chh = sqrtf(1.0f - sh * sh);
    c0 = make_float4(c.x, c.y, c.z, sh);
    c1 = make_float4(chh, 2.0f * sh * chh, 0.f, 0.f);
}

// Directions and cap of one tile (one wave); the cap is also returned.
// With kAA the lane also stores its pixel's global delta, and the tile cap
// is widened by the fringe the pixel step adds outside an edge: a pixel is
// touched by a triangle when every edge value exceeds -1/(2 delta) (and the
// miter value, whose cap grows by no more for radii up to pi/2), i.e. within
// asin(1/(2 delta)) of each edge's half-sphere.  For wire frames the fringe
// is 5/4 pixel: a line mask reaches 1/delta from the great circle and half a
// pixel past the segment's cap, so within sqrt(1 + 1/4) < 5/4 pixel of the
// segment (P.fringe holds the factor).
template <bool kAA>
__device__ inline void build_map_tile(const MapParams& P, void* map, int64_t ntiles, int64_t tile, int lane,
                                      float4& c0, float4& c1) {
    int tx = int(tile % P.ntx), ty = int(tile / P.ntx);
    int i = tx * kTile + (lane & (kTile - 1)), j = ty * kTile + (lane >> 3);
    float3 g = f3(0.f, 0.f, 0.f);
    bool ok = false;
    if (i < P.W && j < P.H) ok = pixel_direction(P, i, j, g);
    if (!ok) g = f3(0.f, 0.f, 0.f);
    int64_t q = tile * kTilePix + lane;
    float fringe = 0.0f;
    if (kAA) {
        float delta = tile_pixel_delta(P, tx, ty, i, j, lane, g, ok);
        float* dplane = reinterpret_cast<float*>(reinterpret_cast<char*>(map) + aa_delta_off(P.W, P.H, P.fmt));
        dplane[q] = delta;
        fringe = wave_max(ok ? P.fringe / delta : 0.0f);
    }
    if (P.fmt == VSR_MAP_OCT16) {
        uint32_t w = ok ? oct_encode(g) : kOctInvalid;
        reinterpret_cast<uint32_t*>(map)[q] = w;
        g = oct_decode(w);  // the cap must bound what the rasterizer reads
        ok = (w != kOctInvalid);
    } else {
        float* p = reinterpret_cast<float*>(map);
        int64_t plane = ntiles * kTilePix;
        p[q] = g.x;
        p[plane + q] = g.y;
        p[2 * plane + q] = g.z;
    }
    tile_cap(g, ok, c0, c1);
    if (kAA) dilate_cap(c0, c1, fringe);
    if (lane == 0) {
        MapLayout L = map_layout(P.W, P.H, P.fmt);
        float4* caps = reinterpret_cast<float4*>(reinterpret_cast<char*>(map) + L.caps_off);
        caps[2 * tile] = c0;
        caps[2 * tile + 1] = c1;
    }
}

// One 256-thread block per 16x16 super-tile: wave w builds tile w of the
// 2x2, then one thread bounds the four tile caps by the super-tile cap.
template <bool kAA = false>
__device__ inline void build_map_super(const MapParams& P, void* map, int64_t ntiles, int64_t sidx) {
    __shared__ float4 s_cap[4][2];
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    int64_t tile;
    int tx, ty;
    float4 c0 = make_float4(0.f, 0.f, 1.f, 0.f), c1 = make_float4(1.f, 0.f, kCapEmpty, 0.f);
    if (super_tile_of(sidx, w, P.ntx, P.nty, tile, tx, ty)) build_map_tile<kAA>(P, map, ntiles, tile, lane, c0, c1);
    if (lane == 0) {
        s_cap[w][0] = c0;
        s_cap[w][1] = c1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        float4 sup0, sup1;
        super_cap_of(s_cap, sup0, sup1);
        float4* sups = const_cast<float4*>(map_sups(map, ntiles, P.fmt));
        sups[2 * sidx] = sup0;
        sups[2 * sidx + 1] = sup1;
    }
}

template <bool kAA>
__global__ __launch_bounds__(256) void k_build_map(MapParams P, void* map, int64_t ntiles) {
    build_map_super<kAA>(P, map, ntiles, blockIdx.x);
}

// Cap of 32x32 block b (2x2 super-tiles) from its super-tile caps; one
// thread per block, after the map kernel.
__device__ inline void block_cap(void* map, int64_t ntiles, int32_t fmt, int32_t ntx, int32_t nty, int64_t b) {
    const int nsx = (ntx + 1) / 2, nsy = (nty + 1) / 2, nbx = (ntx + 3) / 4;
    const int bx = int(b % nbx), by = int(b / nbx);
    const float4* sups = map_sups(map, ntiles, fmt);
    float4 ch[4][2];
    for (int q = 0; q < 4; ++q) {
        const int sx = 2 * bx + (q & 1), sy = 2 * by + (q >> 1);
        if (sx < nsx && sy < nsy) {
            const int64_t si = int64_t(sy) * nsx + sx;
            sup_as_child(sups[2 * si], sups[2 * si + 1], ch[q][0], ch[q][1]);
        } else {
            ch[q][0] = make_float4(0.f, 0.f, 1.f, 0.f);
            ch[q][1] = make_float4(1.f, 0.f, kCapEmpty, 0.f);
        }
    }
    float4 b0, b1;
    super_cap_of(ch, b0, b1);
    float4* blks = const_cast<float4*>(map_blks(map, ntiles, fmt, ntx, nty));
    blks[2 * b] = b0;
    blks[2 * b + 1] = b1;
}

__global__ __launch_bounds__(64) void k_block_caps(void* map, int64_t ntiles, int32_t fmt, int32_t ntx, int32_t nty,
                                                   int64_t nblk) {
    const int64_t b = int64_t(blockIdx.x) * 64 + threadIdx.x;
    if (b < nblk) block_cap(map, ntiles, fmt, ntx, nty, b);
}

__global__ __launch_bounds__(256) void k_map_unpack(const void* map, int32_t fmt, int64_t ntiles, int32_t ntx,
                                                    int32_t W, int32_t H, Rot R, float* out) {
    int lane = threadIdx.x & 63;
    int64_t tile = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
    if (tile >= ntiles) return;
    int tx = int(tile % ntx), ty = int(tile / ntx);
    int i = tx * kTile + (lane & (kTile - 1)), j = ty * kTile + (lane >> 3);
    if (i >= W || j >= H) return;
    float3 g = load_dir(map, fmt, ntiles, tile, lane, R);
    int64_t o = (int64_t(j) * W + i) * 3;
    out[o] = g.x;
    out[o + 1] = g.y;
    out[o + 2] = g.z;
}

hipError_t launch_map_unpack(const void* map, int32_t W, int32_t H, int32_t fmt, const Rot& R, float* out,
                             hipStream_t st) {
    MapLayout L = map_layout(W, H, fmt);
    hipLaunchKernelGGL(k_map_unpack, dim3(unsigned((L.ntiles + 3) / 4)), dim3(256), 0, st, map, fmt, L.ntiles, L.ntx,
                       W, H, R, out);
    return hipGetLastError();
}

hipError_t launch_build_map(const MapParams& P, void* map, bool aa, hipStream_t stream) {
    MapLayout L = map_layout(P.W, P.H, P.fmt);
    if (aa)
        hipLaunchKernelGGL(k_build_map<true>, dim3(unsigned(L.nsup)), dim3(256), 0, stream, P, map, L.ntiles);
    else
        hipLaunchKernelGGL(k_build_map<false>, dim3(unsigned(L.nsup)), dim3(256), 0, stream, P, map, L.ntiles);
    hipLaunchKernelGGL(k_block_caps, dim3(unsigned((L.nblk + 63) / 64)), dim3(64), 0, stream, map, L.ntiles, P.fmt,
                       L.ntx, L.nty, L.nblk);
    return hipGetLastError();
}

}  // namespace vsr
