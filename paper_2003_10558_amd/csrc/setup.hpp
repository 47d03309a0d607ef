// Per-triangle setup, nearest-first ordering and the cube-map cap index.
//
// k_setup_tris (one thread per triangle, coalesced SoA vertex reads):
//   - the three edge-plane normals A x B, B x C, C x A of section 1.1,
//     each computed from the edge's endpoints in a canonical (lexicographic)
//     order as P x (Q - P) and negated when the order was swapped, so the two
//     triangles sharing an edge get exactly opposite normals;
//   - orientation: the normals are multiplied by sigma = sign(det[A,B,C]) so
//     that either winding covers the inside of its cone, never its antipode;
//   - the hard normal N = (A-B) x (C-B) and d = A.N of section 1.1.4, stored
//     as a unit normal facing away from O and the plane's distance from O;
//   - a depth lower bound for the front-to-back early exit (depth_lb);
//   - the smallest-circle cap of section 1.1.2 (bounding cap of the
//     spherical triangle) and the cube-map cell of its centre at the level
//     matching its radius.
// Then a stable LSD radix sort orders triangles by depth lower bound (its
// top 24 bits; ties keep id order), records are permuted into that order, and a second
// stable radix sort groups them by (depth slice, cell) so that every cell's
// list is itself nearest first.  cell_start[key] is the first entry of
// index key `key`; face_count[s][level*6+face] counts a slice's triangles
// on one cube face of one level.
#pragma once
#include "vsr_internal.h"

namespace vsr {

__device__ inline bool vless(float3 a, float3 b) {
    if (a.x != b.x) return a.x < b.x;
    if (a.y != b.y) return a.y < b.y;
    return a.z < b.z;
}

// Edge-plane normal of edge P->Q, antisymmetric bit for bit: n(P,Q) = -n(Q,P).
__device__ inline float3 edge_normal(float3 P, float3 Q) {
    if (vless(P, Q)) return cross3(P, sub3(Q, P));
    float3 n = cross3(Q, sub3(P, Q));
    return f3(-n.x, -n.y, -n.z);
}

// Cube-map cell of a unit direction at level L.
__device__ inline uint32_t cell_of(float3 s, int L) {
    float ax = fabsf(s.x), ay = fabsf(s.y), az = fabsf(s.z);
    int a;
    float major;
    if (ax >= ay && ax >= az) {
        a = 0;
        major = s.x;
    } else if (ay >= az) {
        a = 1;
        major = s.y;
    } else {
        a = 2;
        major = s.z;
    }
    int face = 2 * a + (major < 0.0f ? 1 : 0);
    float comp[3] = {s.x, s.y, s.z};
    float am = fabsf(major);
    float u = comp[(a + 1) % 3] / am, v = comp[(a + 2) % 3] / am;
    int M = 1 << L;
    int iu = min(M - 1, max(0, int(floorf((u + 1.0f) * 0.5f * M))));
    int iv = min(M - 1, max(0, int(floorf((v + 1.0f) * 0.5f * M))));
    return uint32_t(level_base(L) + int64_t(face) * M * M + int64_t(iv) * M + iu);
}

// ---------------------------------------------- depth lower bound ------
// A bound lb <= every FP32 depth the rasterizer can compute for this
// triangle, so that nearest-first processing may stop once every pixel is
// nearer than the next triangle's lb.  The plane distance d alone is one
// (r = d / (G.N) >= d), but for a triangle seen at an angle the rays that
// cover it meet its plane much further out: r >= d / cos(theta), theta the
// angle from the plane normal to the nearest direction of the triangle's
// cone.  Evaluated in FP32 from the values the rasterizer uses, with every
// rounding bounded and added on the safe side (u = 2^-24):
//   - a stored edge normal n_i = P x (Q - P), rounded and normalised in FP32,
//     deviates from the exact unit normal of the cone's edge by at most
//     (5.25 K + 4) u rad, K = max(|P|, |Q|) |Q - P| / |P x Q| (one rounding
//     of Q - P, three per cross-product component, four for the
//     normalisation); with the FP32 rounding of the rasterizer's n_i . G
//     (8 u) each edge is trusted to eta = (16 K + 32) u, twice that sum;
//   - covered directions then lie in the cone dilated by eta per edge,
//     which near a corner of angle alpha reaches eta / sin(alpha/2),
//     doubled: eta_c = 2 eta / s_min, with sin(alpha/2) bounded below both
//     from the cosine, sqrt((1 - cos alpha)/2), and from the sine,
//     sin(alpha)/2, of the two stored normals that meet there;
//   - cos(theta) is bounded above without angles: the largest of u.v over
//     the vertex directions v and, for each edge whose great circle has the
//     projection of u inside the edge (tested with a 1e-5 allowance, so a
//     borderline edge is counted: its value never falls below the true
//     maximum), sqrt(1 - (u.n_i)^2); plus eta (the edge planes' error),
//     eta_c (the dilation: cos(theta - eta_c) <= cos(theta) + eta_c) and
//     4e-6 for the rounding of these dots, clamped to [cos 1.5, 1];
//   - the FP32 depth d * rcp(G.N) is at least (1 - 3u) r / (1 + 8u r/d)
//     (G.N carries at most 8u of absolute rounding, |G| <= 1 + 2e-6);
// the result is widened by 1e-5 and by 16u for its own rounding.  Never
// below the plane-distance bound d (1 - 2^-16), which is also returned when
// an edge is too ill-conditioned (K u > 1e-3) or a corner too sharp
// (sin(alpha/2) <= 1e-4) for the bound to say more.
__device__ inline float depth_lb(float3 A, float3 B, float3 C, float4 r0, float4 r1, float4 r2, float dist,
                                 float sigma) {
    const float base = dist * (1.0f - 1.0f / 65536.0f);
    const float3 V[3] = {A, B, C};
    const float3 nrm[3] = {f3(r0.x, r0.y, r0.z), f3(r1.x, r1.y, r1.z), f3(r2.x, r2.y, r2.z)};
    float eta = 0.0f;
    for (int i = 0; i < 3; ++i) {
        const float3 P = V[i], Q = V[(i + 1) % 3];
        const float3 D = sub3(Q, P);
        const float3 X = cross3(P, D);
        const float lx = sqrtf(dot3(X, X));
        if (!(lx > 0.0f)) return base;
        const float K = fmaxf(sqrtf(dot3(P, P)), sqrtf(dot3(Q, Q))) * sqrtf(dot3(D, D)) / lx;
        if (!(K * kUlp < 1e-3f)) return base;
        eta = fmaxf(eta, (16.0f * K + 32.0f) * kUlp);
    }
    // smallest corner: A between edges CA (2) and AB (0), B between 0 and 1,
    // C between 1 and 2; the inward normals meet at pi - alpha
    float smin = 1.0f;
    for (int k = 0; k < 3; ++k) {
        const float3 ni = nrm[(k + 2) % 3], nj = nrm[k];
        const float c = dot3(ni, nj);  // -cos(alpha)
        const float s_cos = sqrtf(fmaxf(0.0f, 0.5f * (1.0f + c) - (eta + 4.0f * kUlp)));
        const float3 x = cross3(ni, nj);
        const float s_sin = 0.5f * (sqrtf(dot3(x, x)) - 2.0f * eta - 8.0f * kUlp);
        smin = fminf(smin, fmaxf(s_cos, s_sin));
    }
    if (!(smin > 1e-4f)) return base;
    const float eta_c = 2.0f * eta / smin;
    // unit direction of the stored plane normal
    const float3 nh = f3(r0.w, r1.w, r2.w);
    const float lnh = sqrtf(dot3(nh, nh));
    const float3 u = scale3(nh, 1.0f / lnh);
    bool inside = true;
    for (int i = 0; i < 3; ++i)
        if (dot3(nrm[i], u) < -(eta_c + 8.0f * kUlp)) inside = false;
    float cmax = 1.0f;
    if (!inside) {
        float3 v[3];
        cmax = -1.0f;
        for (int i = 0; i < 3; ++i) {
            v[i] = scale3(V[i], 1.0f / sqrtf(dot3(V[i], V[i])));
            cmax = fmaxf(cmax, dot3(u, v[i]));
        }
        for (int i = 0; i < 3; ++i) {
            const float3 p = v[i], q = v[(i + 1) % 3];
            const float3 so = scale3(nrm[i], sigma);  // along p x q
            const float x = dot3(nrm[i], u);
            const float3 w = sub3(u, scale3(nrm[i], x));  // projection on the great circle
            if (dot3(cross3(p, w), so) >= -1e-5f && dot3(cross3(w, q), so) >= -1e-5f)
                cmax = fmaxf(cmax, sqrtf(fmaxf(0.0f, 1.0f - x * x)));
        }
        cmax += eta + eta_c + 4e-6f;
    }
    const float cos_up = fminf(1.0f, fmaxf(cmax, 0.0707372f));  // cos(1.5) = 0.07073720...
    const float L = dist / (lnh * (1.0f + 2e-6f) * cos_up);
    float lb = L * (1.0f - 3.0f * kUlp) / (1.0f + 8.0f * kUlp * L / dist);
    lb *= (1.0f - 1e-5f) * (1.0f - 16.0f * kUlp);
    return fmaxf(lb, base);
}

__global__ __launch_bounds__(256) void k_setup_tris(const float* __restrict__ xyz, int64_t n,
                                                    float4* __restrict__ rec_id, float4* __restrict__ cap_id,
                                                    uint32_t* __restrict__ key, uint32_t* __restrict__ val,
                                                    uint32_t* __restrict__ bucket) {
    int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= n) return;
    float3 A = f3(xyz[0 * n + t], xyz[1 * n + t], xyz[2 * n + t]);
    float3 B = f3(xyz[3 * n + t], xyz[4 * n + t], xyz[5 * n + t]);
    float3 C = f3(xyz[6 * n + t], xyz[7 * n + t], xyz[8 * n + t]);

    float3 N = cross3(sub3(A, B), sub3(C, B));
    float d = dot3(A, N);
    float lenN = sqrtf(dot3(N, N));
    float lenA = sqrtf(dot3(A, A));
    float3 e0 = edge_normal(A, B), e1 = edge_normal(B, C), e2 = edge_normal(C, A);
    float l0 = dot3(e0, e0), l1 = dot3(e1, e1), l2 = dot3(e2, e2);
    // det[A,B,C] = -A.N: cull when the plane passes (to FP32 accuracy) through O
    bool live = fabsf(d) > 1e-7f * lenA * lenN && l0 > 0.0f && l1 > 0.0f && l2 > 0.0f;

    float4 r0, r1, r2, r3, c0, c1;
    uint32_t bkt = uint32_t(kNumBuckets);
    float lb = __int_as_float(0x7F800000);  // +inf: sorted last
    if (live) {
        float sigma = d < 0.0f ? 1.0f : -1.0f;  // sign(det[A,B,C])
        float s0 = sigma / sqrtf(l0), s1 = sigma / sqrtf(l1), s2 = sigma / sqrtf(l2);
        float sn = (d > 0.0f ? 1.0f : -1.0f) / lenN;
        float dist = fabsf(d) / lenN;
        r0 = make_float4(e0.x * s0, e0.y * s0, e0.z * s0, N.x * sn);
        r1 = make_float4(e1.x * s1, e1.y * s1, e1.z * s1, N.y * sn);
        r2 = make_float4(e2.x * s2, e2.y * s2, e2.z * s2, N.z * sn);
        lb = depth_lb(A, B, C, r0, r1, r2, dist, sigma);
        r3 = make_float4(dist, lb, __uint_as_float(uint32_t(t)), 0.0f);

        // Smallest circle around the sphere-projected vertices (section 1.1.2).
        float3 a = scale3(A, 1.0f / lenA);
        float3 b = scale3(B, 1.0f / sqrtf(dot3(B, B)));
        float3 c = scale3(C, 1.0f / sqrtf(dot3(C, C)));
        float3 dbc = sub3(b, c), dca = sub3(c, a), dab = sub3(a, b);
        float a2 = dot3(dbc, dbc), b2 = dot3(dca, dca), c2 = dot3(dab, dab);
        float ws = a2 * (b2 + c2 - a2), wt = b2 * (c2 + a2 - b2), wp = c2 * (a2 + b2 - c2);
        float3 S;
        if (ws <= 0.0f)
            S = scale3(add3(b, c), 0.5f);
        else if (wt <= 0.0f)
            S = scale3(add3(c, a), 0.5f);
        else if (wp <= 0.0f)
            S = scale3(add3(a, b), 0.5f);
        else
            S = scale3(add3(add3(scale3(a, ws), scale3(b, wt)), scale3(c, wp)), 1.0f / (ws + wt + wp));
        float sl = sqrtf(dot3(S, S));
        const bool degenerate = !(sl > 1e-6f);  // plane of the unit vertices through O
        bool wide = degenerate;
        float rho = kPi, sh_rim = 0.0f;
        if (!wide) {
            S = scale3(S, 1.0f / sl);
            // radius from the actual vertex chords, robust to rounding in S
            float3 da = sub3(a, S), db = sub3(b, S), dc = sub3(c, S);
            float ch2 = fmaxf(dot3(da, da), fmaxf(dot3(db, db), dot3(dc, dc)));
            sh_rim = fminf(1.0f, 0.5f * sqrtf(ch2));  // sine of half the exact radius (miter rim)
            rho = 2.0f * asinf(sh_rim);
            rho = rho * (1.0f + kCapRelMargin) + kCapAbsMargin;
            wide = !(rho < kHalfPi);
        }
        int L = 0;
        if (!wide) {
            float sh, chh;
            sincosf(0.5f * rho, &sh, &chh);
            c0 = make_float4(S.x, S.y, S.z, sh);
            c1 = make_float4(chh, sinf(rho), 0.0f, sh_rim);
            // finest level whose cell radius bound (pi/4)/2^L still covers rho
            while (L < kMaxLevel && rho <= kQuarterPi / float(1 << (L + 1))) ++L;
            if (rho > kQuarterPi) L = 0;
            bkt = cell_of(S, L);
        } else {
            // no culling; the centre and rim still define the miter unless degenerate
            c0 = degenerate ? make_float4(0.0f, 0.0f, 1.0f, 1.0f) : make_float4(S.x, S.y, S.z, 1.0f);
            c1 = make_float4(0.0f, 1.0f, kCapWide, sh_rim);
            bkt = uint32_t(level_base(0));  // level 0, face 0: every tile looks at level 0
        }
    } else {
        r0 = r1 = r2 = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        r3 = make_float4(0.0f, lb, __uint_as_float(uint32_t(t)), 0.0f);
        c0 = make_float4(0.0f, 0.0f, 1.0f, 0.0f);
        c1 = make_float4(1.0f, 0.0f, kCapEmpty, 0.0f);
    }
    rec_id[4 * t + 0] = r0;
    rec_id[4 * t + 1] = r1;
    rec_id[4 * t + 2] = r2;
    rec_id[4 * t + 3] = r3;
    cap_id[2 * t + 0] = c0;
    cap_id[2 * t + 1] = c1;
    key[t] = depth_key(lb);
    val[t] = uint32_t(t);
    bucket[t] = bkt;
}

// ------------------------------------------------ stable LSD radix sort --
// Blocks of kSortBlock consecutive keys; per pass: per-block digit
// histogram, exclusive scans over blocks per digit (and over the digit
// totals, inside the scatter), stable scatter.

__global__ __launch_bounds__(kSortThreads) void k_rs_hist(const uint32_t* __restrict__ keys, int64_t n, int shift,
                                                          uint32_t* __restrict__ hist, int64_t nblocks) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    int64_t base = int64_t(blockIdx.x) * kSortBlock;
    for (int r = 0; r < kSortItems; ++r) {
        int64_t i = base + r * kSortThreads + threadIdx.x;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[int64_t(threadIdx.x) * nblocks + blockIdx.x] = h[threadIdx.x];
}

// Exclusive scan of one digit's row of per-block counts (one workgroup per
// digit); the row total goes to tot[digit].
__global__ __launch_bounds__(256) void k_rs_scan_rows(uint32_t* __restrict__ hist, int64_t nblocks,
                                                      uint32_t* __restrict__ tot) {
    __shared__ uint32_t part[256];
    uint32_t* a = hist + int64_t(blockIdx.x) * nblocks;
    int64_t per = (nblocks + 255) / 256;
    int64_t b = int64_t(threadIdx.x) * per, e = min(nblocks, b + per);
    uint32_t s = 0;
    for (int64_t i = b; i < e; ++i) s += a[i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        uint32_t v = threadIdx.x >= unsigned(o) ? part[threadIdx.x - o] : 0u;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    uint32_t run = threadIdx.x > 0 ? part[threadIdx.x - 1] : 0u;
    for (int64_t i = b; i < e; ++i) {
        uint32_t v = a[i];
        a[i] = run;
        run += v;
    }
    if (threadIdx.x == 255) tot[blockIdx.x] = part[255];
}

// Stable scatter of one block: each element's rank within its digit comes
// from ballots (8 rounds of 256 in input order), the block is then staged in
// LDS sorted by digit, and written out so that consecutive threads store
// consecutive positions of one digit's run (one coalesced segment per digit
// instead of one 4-byte store per element).
__global__ __launch_bounds__(kSortThreads) void k_rs_scatter(const uint32_t* __restrict__ kin,
                                                             const uint32_t* __restrict__ vin,
                                                             uint32_t* __restrict__ kout, uint32_t* __restrict__ vout,
                                                             int64_t n, int shift, const uint32_t* __restrict__ offs,
                                                             int64_t nblocks, const uint32_t* __restrict__ tot) {
    __shared__ uint32_t gbase[256];  // output position of this block's first element of each digit
    __shared__ uint32_t lrun[256];   // block-local count of each digit, then its first slot in the stage
    __shared__ uint32_t wcnt[kSortThreads / 64][256];
    __shared__ uint32_t sk[kSortBlock], sv[kSortBlock];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    // first position of digit tid: exclusive scan of the 256 digit totals
    // (every workgroup scans them itself: no separate launch)
    uint32_t x = tot[tid];
    const uint32_t own = x;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) wcnt[0][wave] = x;
    __syncthreads();
    uint32_t first = x - own;
    for (int q = 0; q < wave; ++q) first += wcnt[0][q];
    __syncthreads();
    gbase[tid] = first + offs[int64_t(tid) * nblocks + blockIdx.x];
    lrun[tid] = 0;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int64_t base = int64_t(blockIdx.x) * kSortBlock;
    uint32_t kk[kSortItems], vv[kSortItems], pos[kSortItems];
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        for (int w = 0; w < kSortThreads / 64; ++w) wcnt[w][tid] = 0;
        __syncthreads();
        const int64_t i = base + r * kSortThreads + tid;
        const bool valid = i < n;
        const uint32_t k = valid ? kin[i] : 0u, v = valid ? vin[i] : 0u;
        const uint32_t dg = (k >> shift) & 255u;
        uint64_t same = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            uint64_t m = __ballot((dg >> bit) & 1u);
            same &= ((dg >> bit) & 1u) ? m : ~m;
        }
        const uint32_t rank = (uint32_t)__popcll(same & lt);
        if (valid && rank == 0) wcnt[wave][dg] = (uint32_t)__popcll(same);
        __syncthreads();
        uint32_t p = 0xFFFFFFFFu;  // rank within the digit over the block so far
        if (valid) {
            p = lrun[dg] + rank;
            for (int w = 0; w < wave; ++w) p += wcnt[w][dg];
        }
        kk[r] = k;
        vv[r] = v;
        pos[r] = p;
        __syncthreads();
        uint32_t add = 0;
        for (int w = 0; w < kSortThreads / 64; ++w) add += wcnt[w][tid];
        lrun[tid] += add;
    }
    __syncthreads();
    // first stage slot of each digit: exclusive scan of the block's counts
    const uint32_t c = lrun[tid];
    x = c;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) wcnt[0][wave] = x;
    __syncthreads();
    uint32_t start = x - c;
    for (int q = 0; q < wave; ++q) start += wcnt[0][q];
    lrun[tid] = start;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        if (pos[r] != 0xFFFFFFFFu) {
            const uint32_t q = lrun[(kk[r] >> shift) & 255u] + pos[r];
            sk[q] = kk[r];
            sv[q] = vv[r];
        }
    }
    __syncthreads();
    const uint32_t nvalid = uint32_t(min(int64_t(kSortBlock), n - base));
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        const uint32_t q = uint32_t(r * kSortThreads + tid);
        if (q < nvalid) {
            const uint32_t k = sk[q];
            const uint32_t d = (k >> shift) & 255u;
            const uint32_t o = gbase[d] + (q - lrun[d]);
            kout[o] = k;
            vout[o] = sv[q];
        }
    }
}

// Sort (key, val) pairs of length n on `bits` low key bits (multiple of 8).
// Returns which buffer pair holds the result: false = (ka, va), true = (kb, vb).
static hipError_t radix_sort(uint32_t* ka, uint32_t* va, uint32_t* kb, uint32_t* vb, uint32_t* hist, int64_t n,
                             int bits, bool* in_b, hipStream_t st) {
    int64_t nb = (n + kSortBlock - 1) / kSortBlock;
    bool b = false;
    for (int shift = 0; shift < bits; shift += 8) {
        uint32_t *ki = b ? kb : ka, *vi = b ? vb : va, *ko = b ? ka : kb, *vo = b ? va : vb;
        uint32_t* tot = hist + 256 * nb;
        hipLaunchKernelGGL(k_rs_hist, dim3(unsigned(nb)), dim3(kSortThreads), 0, st, ki, n, shift, hist, nb);
        hipLaunchKernelGGL(k_rs_scan_rows, dim3(256), dim3(256), 0, st, hist, nb, tot);
        hipLaunchKernelGGL(k_rs_scatter, dim3(unsigned(nb)), dim3(kSortThreads), 0, st, ki, vi, ko, vo, n, shift,
                           hist, nb, tot);
        b = !b;
    }
    *in_b = b;
    return hipGetLastError();
}

// Permute records and caps into nearest-first order; prepare the cell sort.
// Depth buckets: ranks are grouped into 2^bucket_shift(n) consecutive ranks
// (at most 256 buckets).  Every record's fourth word of r3 receives the depth
// lower bound of the first rank of its bucket, floored to its sort key
// (depth_key_floor), which bounds the lower bound of every triangle in that
// bucket and in all later ones; the permutation writes it with the record
// (read from the bucket's first source record).
__global__ __launch_bounds__(256) void k_permute(const uint32_t* __restrict__ order_ids, int64_t n, int shift,
                                                 const float4* __restrict__ rec_id, const float4* __restrict__ cap_id,
                                                 const uint32_t* __restrict__ bucket, float4* __restrict__ rec,
                                                 float4* __restrict__ cap, float4* __restrict__ rcap,
                                                 uint32_t* __restrict__ order, uint32_t* __restrict__ key2,
                                                 uint32_t* __restrict__ val2) {
    int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r >= n) return;
    uint32_t id = order_ids[r];
    const uint32_t first_id = order_ids[(r >> shift) << shift];
#pragma unroll
    for (int q = 0; q < 3; ++q) rec[4 * r + q] = rec_id[4 * int64_t(id) + q];
    float4 r3 = rec_id[4 * int64_t(id) + 3];
    r3.w = depth_key_floor(rec_id[4 * int64_t(first_id) + 3].y);
    rec[4 * r + 3] = r3;
    const float4 c0 = cap_id[2 * int64_t(id) + 0], c1 = cap_id[2 * int64_t(id) + 1];
    cap[2 * r + 0] = c0;
    cap[2 * r + 1] = c1;
    // the binning cap (as in the cell-ordered copy), in rank order
    rcap[r] = make_float4(c0.x, c0.y, c0.z, (c1.z == kCapWide) ? kBinWide : c0.w);
    order[r] = id;
    uint32_t b = bucket[id];
    key2[r] = b == uint32_t(kNumBuckets) ? uint32_t(kIndexKeys)
                                         : uint32_t(int64_t(slice_of(n, r)) * kNumBuckets + b);
    val2[r] = uint32_t(r);
}

// Cell-ordered copies: cell_list[k] = rank of the k-th entry and its
// binning record (cap + edge normals).
__device__ inline void cell_record(int64_t k, const uint32_t* __restrict__ ranks, const float4* __restrict__ rec,
                                   const float4* __restrict__ cap, uint32_t* __restrict__ cell_list,
                                   float4* __restrict__ bincap, float4* __restrict__ binnrm) {
    uint32_t r = ranks[k];
    cell_list[k] = r;
    float4 c0 = cap[2 * int64_t(r)], c1 = cap[2 * int64_t(r) + 1];
    float4 r0 = rec[4 * int64_t(r)], r1 = rec[4 * int64_t(r) + 1], r2 = rec[4 * int64_t(r) + 2];
    float sh = (c1.z == kCapWide) ? kBinWide : c0.w;
    bincap[k] = make_float4(c0.x, c0.y, c0.z, sh);
    binnrm[3 * k + 0] = make_float4(r0.x, r0.y, r0.z, __uint_as_float(r));
    binnrm[3 * k + 1] = make_float4(r1.x, r1.y, r1.z, 0.0f);
    binnrm[3 * k + 2] = make_float4(r2.x, r2.y, r2.z, 0.0f);
}

// cell_start[b] = first position whose index key is >= b (lower bound).
__device__ inline void cell_start_of(int64_t b, const uint32_t* __restrict__ sorted_bucket, int64_t n,
                                     uint32_t* __restrict__ cell_start) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (int64_t(sorted_bucket[mid]) < b)
            lo = mid + 1;
        else
            hi = mid;
    }
    cell_start[b] = uint32_t(lo);
}

constexpr unsigned kCellStartBlocks = unsigned((kIndexKeys + 1 + 255) / 256);

// The cap index from the cell-sorted pairs, in one launch: workgroups
// [0, kCellStartBlocks) find the cell starts (latency-bound binary
// searches), the rest gather the cell-ordered binning records (bandwidth-
// bound), so the two overlap.
__global__ __launch_bounds__(256) void k_cell_index(const uint32_t* __restrict__ sorted_bucket,
                                                    const uint32_t* __restrict__ ranks, int64_t n,
                                                    const float4* __restrict__ rec, const float4* __restrict__ cap,
                                                    uint32_t* __restrict__ cell_start, uint32_t* __restrict__ cell_list,
                                                    float4* __restrict__ bincap, float4* __restrict__ binnrm) {
    if (blockIdx.x < kCellStartBlocks) {
        const int64_t b = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
        if (b <= kIndexKeys) cell_start_of(b, sorted_bucket, n, cell_start);
    } else {
        const int64_t k = int64_t(blockIdx.x - kCellStartBlocks) * blockDim.x + threadIdx.x;
        if (k < n) cell_record(k, ranks, rec, cap, cell_list, bincap, binnrm);
    }
}

// Triangles of slice s on cube face `face` of level L (p = L*6 + face).
__global__ __launch_bounds__(64) void k_face_count(const uint32_t* __restrict__ cell_start,
                                                   uint32_t* __restrict__ face_count) {
    int s = blockIdx.x, p = threadIdx.x;
    uint32_t c = 0;
    if (p < 6 * kLevels) {
        int L = p / 6, face = p % 6, M = 1 << L;
        int64_t fb = int64_t(s) * kNumBuckets + level_base(L) + int64_t(face) * M * M;
        c = cell_start[fb + int64_t(M) * M] - cell_start[fb];
    }
    face_count[s * 64 + p] = c;
}

// Section 1.3 particles as primitives of the same setup: position P and
// radius r (pr = float[4][n]).  The record holds no edge planes (zero
// normals pass every edge test of the binner), the plane through P with
// normal P_hat (where texture coordinates live and depth is measured), and
// |P| as depth lower bound; the cap is the sphere's silhouette cone,
// sin(rho) = r/|P|, with the exact half-angle sine in its last word.  A
// particle with r <= 0 or containing O covers nothing.
__global__ __launch_bounds__(256) void k_setup_particles(const float* __restrict__ pr, int64_t n,
                                                         float4* __restrict__ rec_id, float4* __restrict__ cap_id,
                                                         uint32_t* __restrict__ key, uint32_t* __restrict__ val,
                                                         uint32_t* __restrict__ bucket) {
    int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= n) return;
    float3 P = f3(pr[0 * n + t], pr[1 * n + t], pr[2 * n + t]);
    float r = pr[3 * n + t];
    float d = sqrtf(dot3(P, P));
    bool live = r > 0.0f && d > r;
    float4 r0, r1, r2, r3, c0, c1;
    uint32_t bkt = uint32_t(kNumBuckets);
    float lb = __int_as_float(0x7F800000);
    if (live) {
        float3 Ph = scale3(P, 1.0f / d);
        lb = d * (1.0f - 1.0f / 65536.0f);
        r0 = make_float4(0.0f, 0.0f, 0.0f, Ph.x);
        r1 = make_float4(0.0f, 0.0f, 0.0f, Ph.y);
        r2 = make_float4(0.0f, 0.0f, 0.0f, Ph.z);
        r3 = make_float4(d, lb, __uint_as_float(uint32_t(t)), 0.0f);
        float s = fminf(1.0f, r / d);
        float sh_rim = sinf(0.5f * asinf(s));
        float rho = 2.0f * asinf(sh_rim);
        rho = rho * (1.0f + kCapRelMargin) + kCapAbsMargin;
        int L = 0;
        if (rho < kHalfPi) {
            float sh, chh;
            sincosf(0.5f * rho, &sh, &chh);
            c0 = make_float4(Ph.x, Ph.y, Ph.z, sh);
            c1 = make_float4(chh, sinf(rho), 0.0f, sh_rim);
            while (L < kMaxLevel && rho <= kQuarterPi / float(1 << (L + 1))) ++L;
            if (rho > kQuarterPi) L = 0;
            bkt = cell_of(Ph, L);
        } else {
            c0 = make_float4(Ph.x, Ph.y, Ph.z, 1.0f);
            c1 = make_float4(0.0f, 1.0f, kCapWide, sh_rim);
            bkt = uint32_t(level_base(0));
        }
    } else {
        r0 = r1 = r2 = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        r3 = make_float4(0.0f, lb, __uint_as_float(uint32_t(t)), 0.0f);
        c0 = make_float4(0.0f, 0.0f, 1.0f, 0.0f);
        c1 = make_float4(1.0f, 0.0f, kCapEmpty, 0.0f);
    }
    rec_id[4 * t + 0] = r0;
    rec_id[4 * t + 1] = r1;
    rec_id[4 * t + 2] = r2;
    rec_id[4 * t + 3] = r3;
    cap_id[2 * t + 0] = c0;
    cap_id[2 * t + 1] = c1;
    key[t] = depth_key(lb);
    val[t] = uint32_t(t);
    bucket[t] = bkt;
}

// Setup of n primitives: `prims` writes the per-primitive records (id
// order), then the nearest-first order, depth buckets and cap index are
// built the same way for every kind of primitive.
template <typename Prims>
hipError_t launch_setup_common(int64_t n, void* setup, hipStream_t st, Prims prims) {
    SetupLayout L = setup_layout(n);
    char* base = reinterpret_cast<char*>(setup);
    auto U = [&](int64_t off) { return reinterpret_cast<uint32_t*>(base + off); };
    auto F4 = [&](int64_t off) { return reinterpret_cast<float4*>(base + off); };
    if (n > 0) {
        unsigned blocks = unsigned((n + 255) / 256);
        prims(blocks, F4(L.rec_id_off), F4(L.cap_id_off), U(L.key_a_off), U(L.val_a_off), U(L.bucket_off));
        bool in_b = false;
        hipError_t e = radix_sort(U(L.key_a_off), U(L.val_a_off), U(L.key_b_off), U(L.val_b_off), U(L.hist_off), n,
                                  kDepthKeyBits, &in_b, st);
        if (e != hipSuccess) return e;
        uint32_t* ids = in_b ? U(L.val_b_off) : U(L.val_a_off);
        // the cell sort writes into the pair not holding ids
        uint32_t* k2 = in_b ? U(L.key_a_off) : U(L.key_b_off);
        uint32_t* v2 = in_b ? U(L.val_a_off) : U(L.val_b_off);
        hipLaunchKernelGGL(k_permute, dim3(blocks), dim3(256), 0, st, ids, n, bucket_shift(n), F4(L.rec_id_off),
                           F4(L.cap_id_off), U(L.bucket_off), F4(L.rec_off), F4(L.cap_off), F4(L.rcap_off),
                           U(L.order_off), k2, v2);
        // ids are no longer needed: the other pair is free scratch
        uint32_t* k3 = in_b ? U(L.key_b_off) : U(L.key_a_off);
        uint32_t* v3 = in_b ? U(L.val_b_off) : U(L.val_a_off);
        bool in3 = false;
        e = radix_sort(k2, v2, k3, v3, U(L.hist_off), n, 24, &in3, st);
        if (e != hipSuccess) return e;
        uint32_t* sk = in3 ? k3 : k2;
        uint32_t* sv = in3 ? v3 : v2;
        hipLaunchKernelGGL(k_cell_index, dim3(kCellStartBlocks + blocks), dim3(256), 0, st, sk, sv, n, F4(L.rec_off),
                           F4(L.cap_off), U(L.cell_start_off), U(L.cell_list_off), F4(L.bincap_off),
                           F4(L.binnrm_off));
    } else {
        hipLaunchKernelGGL(k_cell_index, dim3(kCellStartBlocks), dim3(256), 0, st, U(L.key_a_off), U(L.val_a_off),
                           int64_t(0), F4(L.rec_off), F4(L.cap_off), U(L.cell_start_off), U(L.cell_list_off),
                           F4(L.bincap_off), F4(L.binnrm_off));
    }
    hipLaunchKernelGGL(k_face_count, dim3(kSlices), dim3(64), 0, st, U(L.cell_start_off), U(L.face_count_off));
    return hipGetLastError();
}

hipError_t launch_setup(const float* xyz, int64_t n, void* setup, hipStream_t st) {
    return launch_setup_common(n, setup, st,
                               [&](unsigned blocks, float4* rec, float4* cap, uint32_t* key, uint32_t* val,
                                   uint32_t* bkt) {
                                   hipLaunchKernelGGL(k_setup_tris, dim3(blocks), dim3(256), 0, st, xyz, n, rec, cap,
                                                      key, val, bkt);
                               });
}

hipError_t launch_setup_particles(const float* pr, int64_t n, void* setup, hipStream_t st) {
    return launch_setup_common(n, setup, st,
                               [&](unsigned blocks, float4* rec, float4* cap, uint32_t* key, uint32_t* val,
                                   uint32_t* bkt) {
                                   hipLaunchKernelGGL(k_setup_particles, dim3(blocks), dim3(256), 0, st, pr, n, rec,
                                                      cap, key, val, bkt);
                               });
}

}  // namespace vsr
