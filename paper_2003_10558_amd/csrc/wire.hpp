// Aliasing-free wire frame (section 1.2) of the triangles' sides.
//
// One 64-lane wavefront per 8x8 tile of a map built with VSR_MAP_AA_LINES
// (caps widened by 5/4 pixel), over the ordinary bins of the triangle scene:
// every side that can draw into a tile belongs to a listed triangle.  For a
// side P->Q the lane forms the line step of its great circle with the global
// delta, h = 1 - min(|n.g| delta, 1), and the pixel step of the cap around
// the segment (centre L = |P_hat + Q_hat|, cos of its radius |(P_hat +
// Q_hat)/2|), written through the chord |g - L| and divided by sin of the
// radius like the miter value; the side's mask is the smaller of the two.
// Lines do not hide each other: the pixel keeps the largest mask and the
// triangle it came from (ties: the lower id).
//
// The sides' caps are prepared once per scene (vsr_setup_wire) into a
// rank-ordered array beside the setup records, 64 bytes per triangle:
// (L_0, a_0), (L_1, a_1), (L_2, a_2), (b_0, b_1, b_2, id).  Records are
// staged eight triangles at a time: lanes 8t + e (e < 3) hold edge normal e
// with b_e in its fourth word, lanes 8t + 3 + e side e's cap, lane 8t + 6
// the word with the id.
#pragma once
#include "aa.hpp"

namespace vsr {

struct WireArgs {
    const void* map;
    int64_t ntiles;
    int32_t fmt, depth, W, H, ntx;
    const void* setup;
    const float4* wire;  // 4 per rank (vsr_setup_wire)
    int64_t n;
    const void* bins;
    float* cov;
    uint32_t* dom;
    unsigned long long* stats;  // optional: mask evaluations, (pixel, triangle) pairs with a mask > 0, tiles
    Rot rot;

    __device__ inline void globalize() {
        map = to_global(map);
        setup = to_global(setup);
        wire = to_global(wire);
        bins = to_global(bins);
        cov = to_global(cov);
        dom = to_global(dom);
        stats = to_global(stats);
    }
};

// Centre of the cap around side P->Q and its constants: value at g =
// a - |g - L|^2 b (see miter_consts); sh is the sine of half the radius.
__device__ inline void side_cap(float3 P, float3 Q, float3& L, float& a, float& b) {
    float3 p = scale3(P, 1.0f / sqrtf(dot3(P, P))), q = scale3(Q, 1.0f / sqrtf(dot3(Q, Q)));
    float3 m = f3(0.5f * (p.x + q.x), 0.5f * (p.y + q.y), 0.5f * (p.z + q.z));
    float ml = sqrtf(dot3(m, m));
    L = ml > 0.0f ? scale3(m, 1.0f / ml) : f3(0.0f, 0.0f, 1.0f);
    float3 c = sub3(p, L);
    float sh = 0.5f * sqrtf(dot3(c, c));
    float2 mc = miter_consts(sh);
    a = mc.x;
    b = mc.y;
}

// Mask of one side at the lane's pixel: n = edge normal (xyz), b in .w;
// cap = (L, a).
__device__ inline float side_mask(float4 n, float4 cap, float3 g, float delta) {
    float e = fmaf(n.z, g.z, fmaf(n.y, g.y, n.x * g.x));
    float h = fmaxf(fmaf(-fabsf(e), delta, 1.0f), 0.0f);
    float dx = g.x - cap.x, dy = g.y - cap.y, dz = g.z - cap.z;
    float q = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
    return fminf(h, gpstep(fmaf(-q, n.w, cap.w), delta));
}

template <bool kStats>
__device__ inline void wire_tile(const WireArgs& A0, int64_t tile, int lane, float4* stg) {
    WireArgs A = A0;
    A.globalize();
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
    float best = 0.0f;
    uint32_t dom = kNoHit;
    unsigned long long n_test = 0, n_frag = 0;

    // the three sides of one triangle: normals (b in .w), caps (L, a), id
    auto visit = [&](float4 n0, float4 n1, float4 n2, float4 k0, float4 k1, float4 k2, uint32_t id) {
        float m = fmaxf(fmaxf(side_mask(n0, k0, g, delta), side_mask(n1, k1, g, delta)), side_mask(n2, k2, g, delta));
        m = has_dir ? m : 0.0f;
        if (m > best || (m == best && m > 0.0f && id < dom)) {
            best = m;
            dom = id;
        }
        if (kStats) {
            ++n_test;
            n_frag += __popcll(__ballot(m > 0.0f));
        }
    };

    float4 tc0, tc1;
    load_tile_cap(caps, tile, A.rot, tc0, tc1);
    // 16x16 bin tiles (VSR_BIN_TILE16) are not read here: every tile then
    // gathers its own candidates, as an overflowed one does
    const bool b16 = reinterpret_cast<const uint32_t*>(bb)[kBinHdrTile] == 16u;
    const uint32_t count = b16 ? uint32_t(A.depth) + 1u : __builtin_amdgcn_readfirstlane(counts[tile]);
    if (count <= uint32_t(A.depth)) {
        const uint32_t* lst = lists + tile * A.depth;
        const uint32_t sub = uint32_t(lane) >> 3, part = uint32_t(lane) & 7u;
        const uint32_t ngroups = (count + 7u) >> 3;
        // this lane's word of triangle `sub` of a group
        auto fetch = [&](uint32_t e) {
            float4 w = make_float4(0.f, 0.f, 0.f, 0.f);
            if (e < count) {
                const int64_t rk = lst[e];
                if (part < 3u) {
                    w = S.rec[4 * rk + part];
                    w.w = reinterpret_cast<const float*>(A.wire + 4 * rk + 3)[part];
                } else if (part < 7u) {
                    w = A.wire[4 * rk + (part - 3u)];
                }
            }
            return w;
        };
        float4 v = fetch(sub);  // group 0; the next group is fetched while one is tested
        for (uint32_t gi = 0; gi < ngroups; ++gi) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            stg[lane] = v;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            if (gi + 1 < ngroups) v = fetch((gi + 1) * 8u + sub);
            const uint32_t nt = min(8u, count - gi * 8u);
            for (uint32_t t = 0; t < nt; ++t) {
                const float4* w = stg + 8 * t;
                visit(w[0], w[1], w[2], w[3], w[4], w[5], __float_as_uint(w[6].w));
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
                const float4* rec = S.rec + 4 * int64_t(rk);
                const float4* wr = A.wire + 4 * int64_t(rk);
                float4 n0 = rec[0], n1 = rec[1], n2 = rec[2], bs = wr[3];
                n0.w = bs.x;
                n1.w = bs.y;
                n2.w = bs.z;
                visit(n0, n1, n2, wr[0], wr[1], wr[2], __float_as_uint(bs.w));
            }
        });
    }
    if (inside) {
        int64_t o = int64_t(j) * A.W + i;
        A.cov[o] = best;
        A.dom[o] = dom;
    }
    const unsigned long long npix = kStats ? (unsigned long long)__popcll(__ballot(has_dir)) : 0ull;
    if (kStats && lane == 0) {
        atomicAdd(&A.stats[0], n_test * npix);
        atomicAdd(&A.stats[1], n_frag);
        atomicAdd(&A.stats[3], 1ull);
    }
}

// Side caps of every triangle, stored in rank order (once per scene, after
// the setup).  First the rank of every id is scattered into the scratch tail
// of the wire buffer (rank_of[order[r]] = r); then one thread per triangle
// id reads the [9][n] vertex rows coalesced and writes its 64-byte entry at
// the triangle's rank (one whole line).  The scatter lives here rather than
// in the setup, which runs for every frame of a changing scene and would pay
// for it whether wire frames are drawn or not.
__global__ __launch_bounds__(256) void k_wire_rank(const uint32_t* __restrict__ order, int64_t n,
                                                   uint32_t* __restrict__ rank_of) {
    const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r < n) rank_of[order[r]] = uint32_t(r);
}

__global__ __launch_bounds__(256) void k_setup_wire(const uint32_t* __restrict__ rank_of,
                                                    const float* __restrict__ xyz, int64_t n,
                                                    float4* __restrict__ wire) {
    const int64_t id = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (id >= n) return;
    const int64_t rk = rank_of[id];
    float3 V[3];
    for (int c = 0; c < 3; ++c) V[c] = f3(xyz[(3 * c + 0) * n + id], xyz[(3 * c + 1) * n + id], xyz[(3 * c + 2) * n + id]);
    float b[3];
    for (int e = 0; e < 3; ++e) {
        float3 L;
        float a;
        side_cap(V[e], V[e == 2 ? 0 : e + 1], L, a, b[e]);
        wire[4 * rk + e] = make_float4(L.x, L.y, L.z, a);
    }
    wire[4 * rk + 3] = make_float4(b[0], b[1], b[2], __uint_as_float(uint32_t(id)));
}

// Bytes of the side caps (64 per triangle) and of the scratch tail (4 per
// triangle) of a wire buffer.
inline int64_t wire_caps_bytes(int64_t n) { return align256(n * 64 > 0 ? n * 64 : 256); }
inline int64_t wire_total_bytes(int64_t n) { return wire_caps_bytes(n) + align256(n * 4 > 0 ? n * 4 : 256); }

hipError_t launch_setup_wire(const void* setup, const float* xyz, int64_t n, void* wire, hipStream_t st) {
    if (n > 0) {
        const uint32_t* order =
            reinterpret_cast<const uint32_t*>(static_cast<const char*>(setup) + setup_layout(n).order_off);
        uint32_t* rank_of = reinterpret_cast<uint32_t*>(static_cast<char*>(wire) + wire_caps_bytes(n));
        const unsigned blocks = unsigned((n + 255) / 256);
        hipLaunchKernelGGL(k_wire_rank, dim3(blocks), dim3(256), 0, st, order, n, rank_of);
        hipLaunchKernelGGL(k_setup_wire, dim3(blocks), dim3(256), 0, st, rank_of, xyz, n,
                           reinterpret_cast<float4*>(wire));
    }
    return hipGetLastError();
}

template <bool kStats>
__global__ __launch_bounds__(256) void k_wire(WireArgs A) {
    __shared__ float4 s_stage[4][64];
    int w = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    // workgroups of 4 consecutive tiles, ntx tiles per row
    int64_t tile = band_remap(blockIdx.x, gridDim.x, max(int64_t(1), int64_t(A.ntx) * kBandPx / (4 * kTile))) * 4 + w;
    if (tile >= A.ntiles) return;
    wire_tile<kStats>(A, tile, threadIdx.x & 63, s_stage[w]);
}

hipError_t launch_wire(const void* map, int32_t W, int32_t H, int32_t fmt, const Rot& R, const void* setup,
                       const void* wire, int64_t n, const void* bins, int32_t depth, float* cov, uint32_t* dom,
                       unsigned long long* stats, hipStream_t st) {
    MapLayout ML = map_layout(W, H, fmt);
    WireArgs A;
    A.map = map;
    A.ntiles = ML.ntiles;
    A.fmt = fmt;
    A.depth = depth;
    A.W = W;
    A.H = H;
    A.ntx = ML.ntx;
    A.setup = setup;
    A.wire = reinterpret_cast<const float4*>(wire);
    A.n = n;
    A.bins = bins;
    A.cov = cov;
    A.dom = dom;
    A.stats = stats;
    A.rot = R;
    const dim3 grid = dim3(unsigned((ML.ntiles + 3) / 4)), block = dim3(256);
    if (stats) {
        hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, reinterpret_cast<uint32_t*>(stats), int64_t(8));
        hipLaunchKernelGGL(k_wire<true>, grid, block, 0, st, A);
    } else {
        hipLaunchKernelGGL(k_wire<false>, grid, block, 0, st, A);
    }
    return hipGetLastError();
}

}  // namespace vsr
