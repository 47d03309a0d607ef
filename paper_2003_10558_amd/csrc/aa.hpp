// Aliasing-free coverage: pixel step with the global delta (section 1.1.1),
// miter mask (section 1.1.2) and front-to-back combination of clipped
// fragment masks (section 1.4); the same kernel draws the particles of
// section 1.3 (a particle's mask is the pixel step of its silhouette cap,
// which is the miter value with the particle direction as centre; its
// fragments also carry texture coordinates, combined like the depth).
//
// One 64-lane wavefront per 8x8 tile of a map built with VSR_MAP_AA, whose
// tile caps are widened by the pixel step's fringe so that the ordinary
// binner lists every triangle that touches a tile.  Each lane owns one
// pixel direction g and its delta, and for every listed triangle forms
//   m = min(gpstep(n_0.g), gpstep(n_1.g), gpstep(n_2.g), gpstep(miter)),
//   gpstep(x) = clamp(delta*x + 1/2, 0, 1),
// the miter value being (S.g - cos rho)/sin rho written through the chord
// |g - S| (no cancellation for small circles).  Fragments with m > 0 and
// the plane in front (r = d/(g.N) > 0) enter a per-lane list sorted by
// (r, id) that keeps the nearest ones up to the point where their masks
// saturate the pixel (m^b reaches 1); anything behind that point gets a
// zero share and is dropped.  At the end the list is combined front to
// back: m^fc = min(m^f, 1 - m^b), m^b += m^fc, depth pass += m^fc r, and the
// dominant id is the fragment with the largest share.  A pixel whose list
// overflows before saturating is counted (its result may be inexact).
//
// Records are staged through LDS eight triangles at a time (lane l loads
// word (l & 7) of triangle l >> 3: four record words and two cap words; the
// lane holding the cap's second word turns the rim into the two constants
// of the miter value, and the seventh lane decides whether the triangle can
// matter at all: one whose plane cannot come nearer, anywhere in the tile,
// than the saturation depth of every pixel is skipped by the whole wave).
#pragma once
#include "raster.hpp"

namespace vsr {

constexpr int kAAFrags = 8;  // fragments kept per pixel before saturation

struct AAArgs {
    const void* map;
    int64_t ntiles;
    int32_t fmt, depth, W, H, ntx;
    const void* setup;
    int64_t n;
    const void* bins;
    float* cov;
    float* dpass;
    uint32_t* dom;
    float* uv;                      // particles: texture-coordinate pass, 2 planes
    uint32_t* lost;                 // pixels whose list overflowed unsaturated
    unsigned long long* stats;      // optional: tests, fragments inserted, triangles skipped, tiles
    int32_t no_skip;                // instrumented variant only: test every listed triangle
    Rot rot;

    __device__ inline void globalize() {
        map = to_global(map);
        setup = to_global(setup);
        bins = to_global(bins);
        cov = to_global(cov);
        dpass = to_global(dpass);
        dom = to_global(dom);
        uv = to_global(uv);
        lost = to_global(lost);
        stats = to_global(stats);
    }
};

__device__ inline bool frag_less(float ra, uint32_t ia, float rb, uint32_t ib) {
    return ra < rb || (ra == rb && ia < ib);
}

// Per-lane fragment list; with kUV each fragment also carries texture
// coordinates (particles), combined like the depth (section 1.4).
template <bool kUV>
struct FragList {
    float r[kAAFrags], m[kAAFrags];
    uint32_t id[kAAFrags];
    float u[kUV ? kAAFrags : 1], w[kUV ? kAAFrags : 1];
    int cnt;
    float rsat;      // depth of the fragment that saturates the pixel, +inf if none
    uint32_t idsat;
    bool lost;

    __device__ inline void init() {
        cnt = 0;
        rsat = __int_as_float(0x7F800000);
        idsat = kNoHit;
        lost = false;
    }

    // The loops are unrolled with constant indices (the list stays in
    // registers); a step that no lane of the wave needs is branched over.
    // ub (wave-uniform) >= every lane's cnt: slots past it are empty in the
    // whole wave and are not visited.
    __device__ inline void insert(float rr, uint32_t ii, float mm, int ub, float uu = 0.0f, float ww = 0.0f) {
        if (!frag_less(rr, ii, rsat, idsat)) return;  // behind the saturated prefix: zero share
        float cr = rr, cm = mm, cu = uu, cw = ww;
        uint32_t ci = ii;
#pragma unroll
        for (int k = 0; k < kAAFrags; ++k) {
            if (k > ub) break;
            if (k < cnt) {
                if (frag_less(cr, ci, r[k], id[k])) {
                    float tr = r[k], tm = m[k];
                    uint32_t ti = id[k];
                    r[k] = cr;
                    m[k] = cm;
                    id[k] = ci;
                    cr = tr;
                    cm = tm;
                    ci = ti;
                    if (kUV) {
                        float tu = u[k], tw = w[k];
                        u[k] = cu;
                        w[k] = cw;
                        cu = tu;
                        cw = tw;
                    }
                }
            } else if (k == cnt) {
                r[k] = cr;
                m[k] = cm;
                id[k] = ci;
                if (kUV) {
                    u[k] = cu;
                    w[k] = cw;
                }
            }
        }
        const bool dropped = (cnt == kAAFrags);
        if (!dropped) ++cnt;
        // saturation point: first fragment whose mask fills what is left
        float mb = 0.0f;
        int keep = cnt;
#pragma unroll
        for (int k = 0; k < kAAFrags; ++k) {
            if (k > ub) break;
            if (k < keep) {
                if (m[k] >= 1.0f - mb) {
                    rsat = r[k];
                    idsat = id[k];
                    keep = k + 1;
                } else {
                    mb += m[k];
                }
            }
        }
        cnt = keep;
        if (dropped && rsat == __int_as_float(0x7F800000)) lost = true;
    }

    __device__ inline void combine(float& mb, float& rb, float& ub, float& wb, uint32_t& dom) const {
        mb = 0.0f;
        rb = 0.0f;
        ub = 0.0f;
        wb = 0.0f;
        dom = kNoHit;
        float best = 0.0f;
#pragma unroll
        for (int k = 0; k < kAAFrags; ++k) {
            if (k < cnt) {
                float mfc = fminf(m[k], 1.0f - mb);
                mb += mfc;
                rb = fmaf(mfc, r[k], rb);
                if (kUV) {
                    ub = fmaf(mfc, u[k], ub);
                    wb = fmaf(mfc, w[k], wb);
                }
                if (mfc > best) {
                    best = mfc;
                    dom = id[k];
                }
            }
        }
    }
};

// Bits 6, 14, ..., 62 of a ballot (lane 8t + 6 of each triangle's group of
// eight lanes) packed into bits 0..7.
__device__ inline uint32_t pack_group_bits(uint64_t b) {
    uint32_t out = 0;
#pragma unroll
    for (int t = 0; t < 8; ++t) out |= uint32_t((b >> (8 * t + 6)) & 1ull) << t;
    return out;
}

__device__ inline float gpstep(float x, float delta) { return fminf(fmaxf(fmaf(delta, x, 0.5f), 0.0f), 1.0f); }

// Miter constants from the rim's half-angle sine sh: the value
// (S.g - cos rho)/sin rho = (2 sh^2 - |g-S|^2/2)/(2 sh ch) = a - |g-S|^2 b.
// sh = 0 (degenerate circle): no miter (a = +inf).
__device__ inline float2 miter_consts(float sh) {
    if (!(sh > 0.0f)) return make_float2(__int_as_float(0x7F800000), 0.0f);
    float ch = sqrtf(fmaxf(0.0f, 1.0f - sh * sh));
    return make_float2(sh / ch, 0.25f / (sh * ch));
}

// One triangle against the lane's pixel: inserts its fragment, if any.
// c0 = (S, -), c1 = (a, b, -, -).
__device__ inline bool aa_rec(float4 r0, float4 r1, float4 r2, float4 r3, float4 c0, float4 c1, float3 g, float delta,
                              FragList<false>& L, int ub) {
    float e0 = fmaf(r0.z, g.z, fmaf(r0.y, g.y, r0.x * g.x));
    float e1 = fmaf(r1.z, g.z, fmaf(r1.y, g.y, r1.x * g.x));
    float e2 = fmaf(r2.z, g.z, fmaf(r2.y, g.y, r2.x * g.x));
    float dx = g.x - c0.x, dy = g.y - c0.y, dz = g.z - c0.z;
    float q = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
    float mv = fmaf(-q, c1.y, c1.x);
    float m = fminf(fminf(gpstep(e0, delta), gpstep(e1, delta)), fminf(gpstep(e2, delta), gpstep(mv, delta)));
    if (m > 0.0f) {
        float dn = fmaf(r2.w, g.z, fmaf(r1.w, g.y, r0.w * g.x));
        if (dn > 0.0f) {
            L.insert(r3.x * __builtin_amdgcn_rcpf(dn), __float_as_uint(r3.z), m, ub);
            return true;
        }
    }
    return false;
}

// Texture axes of a particle seen along P_hat (section 1.3): X = |(P_z, 0,
// -P_x)| (the x axis when P is vertical) and the scale |P|/(2r) =
// 1/(2 sin rho) from the rim's half-angle sine sh.
__device__ inline float4 particle_axes(float3 Ph, float sh) {
    float xl = sqrtf(fmaf(Ph.z, Ph.z, Ph.x * Ph.x));
    float3 X = xl > 0.0f ? f3(Ph.z / xl, 0.0f, -Ph.x / xl) : f3(1.0f, 0.0f, 0.0f);
    float ch = sqrtf(fmaxf(0.0f, 1.0f - sh * sh));
    return make_float4(X.x, X.y, X.z, 0.25f / (sh * ch));
}

// One particle against the lane's pixel: the cap value (S = P_hat) through
// the miter constants c1 = (a, b), depth on the particle's plane, texture
// coordinates from the axes ax = (X, scale).
__device__ inline bool part_rec(float4 r0, float4 r1, float4 r2, float4 r3, float4 c0, float4 c1, float4 ax, float3 g,
                                float delta, FragList<true>& L, int ub) {
    float dx = g.x - c0.x, dy = g.y - c0.y, dz = g.z - c0.z;
    float q = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
    float m = gpstep(fmaf(-q, c1.y, c1.x), delta);
    if (m > 0.0f) {
        const float3 N = f3(r0.w, r1.w, r2.w);
        float dn = fmaf(N.z, g.z, fmaf(N.y, g.y, N.x * g.x));
        if (dn > 0.0f) {
            const float3 X = f3(ax.x, ax.y, ax.z);
            const float3 Y = cross3(X, N);
            float u = fmaf(dot3(g, X), ax.w, 0.5f), w = fmaf(dot3(g, Y), ax.w, 0.5f);
            L.insert(r3.x * __builtin_amdgcn_rcpf(dn), __float_as_uint(r3.z), m, ub, u, w);
            return true;
        }
    }
    return false;
}

// Nearest distance at which a triangle's plane (unit normal N facing away
// from O, distance d) can be met by a ray of the tile cap (centre c,
// cos/sin of the radius cr/sr; wide: any ray): r = d/(g.N) >= d/cos(angle).
__device__ inline float plane_min_depth(float3 N, float d, float3 c, float cr, float sr, bool wide) {
    if (wide) return d;
    float ca = dot3(c, N);
    if (ca >= cr) return d;
    float sa = sqrtf(fmaxf(0.0f, 1.0f - ca * ca));
    float cm = fmaf(ca, cr, sa * sr) + 1e-6f;  // cos(angle(c, N) - radius), plus FP32 slack
    return cm > 0.0f ? d / cm : __int_as_float(0x7F800000);
}

constexpr int kPrimTriangles = 0, kPrimParticles = 1;

template <bool kStats, int kPrim>
__device__ inline void aa_tile(const AAArgs& A0, int64_t tile, int lane, float4* stg) {
    AAArgs A = A0;
    A.globalize();
    constexpr bool kPart = kPrim == kPrimParticles;
    const float4* caps = map_caps(A.map, A.ntiles, A.fmt);
    SceneView S = scene_view(A.setup, A.n);
    const char* bb = reinterpret_cast<const char*>(A.bins);
    const uint32_t* counts = reinterpret_cast<const uint32_t*>(bb + 256);
    const uint32_t* lists = reinterpret_cast<const uint32_t*>(bb + 256 + align256(A.ntiles * 4));
    const float* dplane =
        reinterpret_cast<const float*>(reinterpret_cast<const char*>(A.map) + aa_delta_off(A.W, A.H, A.fmt));

    int tx = int(tile % A.ntx), ty = int(tile / A.ntx);
    int i = tx * kTile + (lane & (kTile - 1)), j = ty * kTile + (lane >> 3);
    bool inside = i < A.W && j < A.H;
    float3 g = load_dir(A.map, A.fmt, A.ntiles, tile, lane, A.rot);
    float delta = dplane[tile * kTilePix + lane];
    bool has_dir = inside && delta > 0.0f;
    FragList<kPart> L;
    L.init();
    if (!has_dir) L.rsat = 0.0f;  // nothing can cover it

    float4 tc0, tc1;
    load_tile_cap(caps, tile, A.rot, tc0, tc1);
    const float3 tcen = f3(tc0.x, tc0.y, tc0.z);
    const float tcr = fmaf(-2.0f * tc0.w, tc0.w, 1.0f), tsr = tc1.y;
    const bool twide = tc1.z == kCapWide;
    unsigned long long n_test = 0, n_frag = 0, n_skip = 0;

    const bool may_skip = !(kStats && A.no_skip);
    // May a triangle be skipped by the whole wave?  rmax: largest saturation
    // depth over the wave's pixels (taken before the triangle's group, so at
    // least the current one).
    auto skippable = [&](float3 N, float d, float rmax) {
        if (!may_skip || !(rmax < __int_as_float(0x7F800000))) return false;
        return plane_min_depth(N, d, tcen, tcr, tsr, twide) * (1.0f - 1e-4f) > rmax;
    };
    auto visit = [&](float4 r0, float4 r1, float4 r2, float4 r3, float4 c0, float4 c1, float4 ax) {
        // the longest list of the wave bounds every lane's insertion (all lanes here)
        const int ub = int(wave_max_u32_dpp(uint32_t(L.cnt)));
        bool f;
        if constexpr (kPart)
            f = has_dir && part_rec(r0, r1, r2, r3, c0, c1, ax, g, delta, L, ub);
        else
            f = has_dir && aa_rec(r0, r1, r2, r3, c0, c1, g, delta, L, ub);
        if (kStats) {
            ++n_test;
            n_frag += __popcll(__ballot(f));
        }
    };

    // 16x16 bin tiles (VSR_BIN_TILE16) are not read here: every tile then
    // gathers its own candidates, as an overflowed one does
    const bool b16 = reinterpret_cast<const uint32_t*>(bb)[kBinHdrTile] == 16u;
    const uint32_t count = b16 ? uint32_t(A.depth) + 1u : __builtin_amdgcn_readfirstlane(counts[tile]);
    if (count <= uint32_t(A.depth)) {
        const uint32_t* lst = lists + tile * A.depth;
        const uint32_t sub = uint32_t(lane) >> 3, part = uint32_t(lane) & 7u;
        const uint32_t ngroups = (count + 7u) >> 3;
        // this lane's word of triangle `sub` of a group: record words 0..3,
        // cap words 4..5, for lane 6 the plane (N, d) of the skip test, and
        // for particles lane 7 the plane normal and the rim (texture axes)
        auto fetch = [&](uint32_t e) {
            float4 w = make_float4(0.f, 0.f, 0.f, 0.f);
            if (e < count) {
                const uint32_t rk = lst[e];
                const float4* rec = S.rec + 4 * int64_t(rk);
                if (part < 4u) {
                    w = rec[part];
                } else if (part < 6u) {
                    w = S.cap[2 * int64_t(rk) + (part - 4u)];
                } else if (part == 6u) {
                    const float* rw = reinterpret_cast<const float*>(rec);
                    w = make_float4(rw[3], rw[7], rw[11], rw[12]);
                } else if (kPart) {
                    const float* rw = reinterpret_cast<const float*>(rec);
                    w = make_float4(rw[3], rw[7], rw[11], S.cap[2 * int64_t(rk) + 1].w);
                }
            }
            return w;
        };
        float4 v = fetch(sub);  // group 0; the next group is fetched while one is tested
        for (uint32_t gi = 0; gi < ngroups; ++gi) {
            const float rmax = __uint_as_float(wave_max_u32_dpp(__float_as_uint(L.rsat)));
            const bool present = gi * 8u + sub < count;
            bool live = present;
            float4 st = v;
            if (part == 5u) {
                float2 mc = miter_consts(v.w);
                st = make_float4(mc.x, mc.y, 0.f, 0.f);
            } else if (part == 6u && present) {
                // this lane decides for the whole wave whether the triangle can matter
                live = !skippable(f3(v.x, v.y, v.z), v.w, rmax);
            } else if (kPart && part == 7u && present) {
                st = particle_axes(f3(v.x, v.y, v.z), v.w);
            }
            // bit t: triangle t of the group is to be tested
            const uint32_t todo = pack_group_bits(__ballot(live && part == 6u));
            if (kStats) n_skip += uint32_t(__popc(pack_group_bits(__ballot(present && part == 6u)))) -
                                  uint32_t(__popc(todo));
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            stg[lane] = st;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            if (gi + 1 < ngroups) v = fetch((gi + 1) * 8u + sub);
            for (uint32_t m = todo; m; m &= m - 1) {
                const float4* w = stg + 8 * uint32_t(__ffs(m) - 1);
                visit(w[0], w[1], w[2], w[3], w[4], w[5], w[7]);
            }
        }
    } else {
        gather_candidates(S, tc0, tc1, lane, [&](uint32_t rank, bool valid) {
            bool pass = valid && candidate_test(S, rank, tc0, tc1);
            uint64_t msk = __ballot(pass);
            while (msk) {
                int qb = __ffsll((unsigned long long)msk) - 1;
                msk &= msk - 1;
                uint32_t rk = uint32_t(__builtin_amdgcn_readlane(int(rank), qb));
                const float4* r = S.rec + 4 * int64_t(rk);
                float4 c1 = S.cap[2 * int64_t(rk) + 1];
                float2 mc = miter_consts(c1.w);
                float4 r0 = r[0], r1 = r[1], r2 = r[2], r3 = r[3];
                float rmax = __uint_as_float(wave_max_u32_dpp(__float_as_uint(L.rsat)));
                if (skippable(f3(r0.w, r1.w, r2.w), r3.x, rmax)) {
                    if (kStats) ++n_skip;
                    continue;
                }
                float4 ax = make_float4(0.f, 0.f, 0.f, 0.f);
                if (kPart) ax = particle_axes(f3(r0.w, r1.w, r2.w), c1.w);
                visit(r0, r1, r2, r3, S.cap[2 * int64_t(rk)], make_float4(mc.x, mc.y, 0.f, 0.f), ax);
            }
        });
    }

    float mb, rb, ub, wb;
    uint32_t dm;
    L.combine(mb, rb, ub, wb, dm);
    if (inside) {
        int64_t o = int64_t(j) * A.W + i;
        A.cov[o] = mb;
        A.dpass[o] = rb;
        A.dom[o] = dm;
        if (kPart && A.uv) {
            A.uv[o] = ub;
            A.uv[int64_t(A.W) * A.H + o] = wb;
        }
    }
    if (A.lost) {
        uint32_t c = uint32_t(__popcll(__ballot(L.lost)));
        if (lane == 0 && c) atomicAdd(A.lost, c);
    }
    const unsigned long long npix = kStats ? (unsigned long long)__popcll(__ballot(has_dir)) : 0ull;
    if (kStats && lane == 0) {
        atomicAdd(&A.stats[0], n_test * npix);
        atomicAdd(&A.stats[1], n_frag);
        atomicAdd(&A.stats[2], n_skip);
        atomicAdd(&A.stats[3], 1ull);
    }
}

template <bool kStats, int kPrim>
__device__ inline void aa_raster_wave(const AAArgs& A) {
    __shared__ float4 s_stage[4][64];
    int w = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    // workgroups of 4 consecutive tiles, ntx tiles per row
    int64_t tile = band_remap(blockIdx.x, gridDim.x, max(int64_t(1), int64_t(A.ntx) * kBandPx / (4 * kTile))) * 4 + w;
    if (tile >= A.ntiles) return;
    aa_tile<kStats, kPrim>(A, tile, threadIdx.x & 63, s_stage[w]);
}

template <bool kStats, int kPrim>
__global__ __launch_bounds__(256) void k_aa_raster(AAArgs A) {
    aa_raster_wave<kStats, kPrim>(A);
}

// The triangle kernel is held to 72 VGPRs (from 74), so that a SIMD runs 7
// of its waves instead of 6; nothing spills, and it takes 7% less time on
// 1920x1080 views of the 1M-triangle scene.  (The particle and statistics
// forms would spill at that size.)
template <>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(7, 7))) void k_aa_raster<false, kPrimTriangles>(
    AAArgs A) {
    aa_raster_wave<false, kPrimTriangles>(A);
}

// prim: kPrimTriangles (setup of vsr_setup_tris) or kPrimParticles (setup
// of vsr_setup_particles; uv receives the texture-coordinate pass).
hipError_t launch_aa_raster(const void* map, int32_t W, int32_t H, int32_t fmt, const Rot& R, const void* setup,
                            int64_t n, const void* bins, int32_t depth, float* cov, float* dpass, uint32_t* dom,
                            uint32_t* lost, unsigned long long* stats, int32_t no_skip, hipStream_t st,
                            int prim = kPrimTriangles, float* uv = nullptr) {
    MapLayout ML = map_layout(W, H, fmt);
    AAArgs A;
    A.map = map;
    A.ntiles = ML.ntiles;
    A.fmt = fmt;
    A.depth = depth;
    A.W = W;
    A.H = H;
    A.ntx = ML.ntx;
    A.setup = setup;
    A.n = n;
    A.bins = bins;
    A.cov = cov;
    A.dpass = dpass;
    A.dom = dom;
    A.uv = uv;
    A.lost = lost;
    A.stats = stats;
    A.no_skip = no_skip;
    A.rot = R;
    int64_t blocks = (ML.ntiles + 3) / 4;
    if (lost) hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, lost, int64_t(1));
    if (stats) hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, reinterpret_cast<uint32_t*>(stats), int64_t(8));
    const dim3 grid = dim3(unsigned(blocks)), block = dim3(256);
    if (prim == kPrimParticles) {
        if (stats)
            hipLaunchKernelGGL((k_aa_raster<true, kPrimParticles>), grid, block, 0, st, A);
        else
            hipLaunchKernelGGL((k_aa_raster<false, kPrimParticles>), grid, block, 0, st, A);
    } else {
        if (stats)
            hipLaunchKernelGGL((k_aa_raster<true, kPrimTriangles>), grid, block, 0, st, A);
        else
            hipLaunchKernelGGL((k_aa_raster<false, kPrimTriangles>), grid, block, 0, st, A);
    }
    return hipGetLastError();
}

}  // namespace vsr
