// Fragment data from barycentric coordinates (vsr_resolve).
//
// Section 1.1.4 (second half): the winner's barycentric vector b of the
// point where the pixel's ray meets the triangle's plane, and vertex data
// interpolated with it (depth is already r; the normal pass is normalised).
// The paper writes b with triple products of the vertices relative to
// P = r G; the same weights follow from the edge planes through O without
// forming P: b_A = G.(B x C) / G.(B x C + C x A + A x B), and likewise for B
// and C.  Here each cross product is taken as P x (Q - P), which keeps FP32
// rounding relative to the triangle's own size.
//
// One 64-lane wavefront per 8x8 tile of the map, one lane per pixel; the
// winner's vertices and data are gathered per pixel (neighbouring pixels
// mostly share a winner, so the gathers hit in cache).  From the [9][T] and
// [3][K][T] arrays one triangle's data spans 9 + 3K memory lines; the
// packed form (vsr_resolve_pack, once per scene) stores each triangle's
// vertices and data in one contiguous row instead.
#pragma once
#include "vsr_internal.h"

namespace vsr {

struct ResolveArgs {
    const void* map;
    int64_t ntiles;
    int32_t fmt, W, H, ntx;
    Rot rot;
    const float* xyz;  // [9][ntri]
    int64_t ntri;
    const uint32_t* tri_id;
    const float* vattr;  // [3][nattr][ntri]
    int32_t nattr, normalize3;
    float* bary;  // [3][H][W] or null
    float* attr;  // [nattr][H][W] or null
    const float* packed;  // rows of `stride` floats per triangle, or null
    int32_t stride, pad_;

    __device__ inline void globalize() {
        map = to_global(map);
        xyz = to_global(xyz);
        tri_id = to_global(tri_id);
        vattr = to_global(vattr);
        bary = to_global(bary);
        attr = to_global(attr);
        packed = to_global(packed);
    }
};

// Floats per triangle row of the packed form: A, B, C (9), then vertex v's
// component k at 9 + v*nattr + k; padded to whole float4.
__host__ __device__ inline int32_t resolve_stride(int32_t nattr) { return (9 + 3 * nattr + 3) & ~3; }

__device__ inline float3 vertex_of(const float* xyz, int64_t ntri, int64_t t, int v) {
    return f3(xyz[(3 * v + 0) * ntri + t], xyz[(3 * v + 1) * ntri + t], xyz[(3 * v + 2) * ntri + t]);
}

template <bool kPacked>
__device__ inline void resolve_tile(const ResolveArgs& A0, int64_t tile, int lane) {
    ResolveArgs A = A0;
    A.globalize();
    const int tx = int(tile % A.ntx), ty = int(tile / A.ntx);
    const int i = tx * kTile + (lane & (kTile - 1)), j = ty * kTile + (lane >> 3);
    if (i >= A.W || j >= A.H) return;
    const int64_t o = int64_t(j) * A.W + i, plane = int64_t(A.W) * A.H;
    const float3 g = load_dir(A.map, A.fmt, A.ntiles, tile, lane, A.rot);
    const uint32_t t = A.tri_id[o];
    float b0 = 0.0f, b1 = 0.0f, b2 = 0.0f;
    bool hit = false;
    if (t != VSR_NO_HIT && int64_t(t) < A.ntri && (g.x != 0.0f || g.y != 0.0f || g.z != 0.0f)) {
        float3 a, b, c;
        if (kPacked) {  // rows start on 16-byte boundaries
            const float4* row = reinterpret_cast<const float4*>(A.packed + int64_t(t) * A.stride);
            const float4 r0 = row[0], r1 = row[1], r2 = row[2];
            a = f3(r0.x, r0.y, r0.z);
            b = f3(r0.w, r1.x, r1.y);
            c = f3(r1.z, r1.w, r2.x);
        } else {
            a = vertex_of(A.xyz, A.ntri, t, 0);
            b = vertex_of(A.xyz, A.ntri, t, 1);
            c = vertex_of(A.xyz, A.ntri, t, 2);
        }
        const float wa = dot3(g, cross3(b, sub3(c, b)));  // G.(B x C)
        const float wb = dot3(g, cross3(c, sub3(a, c)));  // G.(C x A)
        const float wc = dot3(g, cross3(a, sub3(b, a)));  // G.(A x B)
        const float s = wa + wb + wc;
        if (s != 0.0f) {
            b0 = wa / s;
            b1 = wb / s;
            b2 = wc / s;
            hit = true;
        }
    }
    if (A.bary) {
        A.bary[o] = b0;
        A.bary[plane + o] = b1;
        A.bary[2 * plane + o] = b2;
    }
    if (!A.attr) return;
    const int64_t na = A.nattr, n = A.ntri;
    auto interp = [&](int k) -> float {
        if (!hit) return 0.0f;
        float fa, fb, fc;
        if (kPacked) {
            const float* row = A.packed + int64_t(t) * A.stride + 9;
            fa = row[k];
            fb = row[na + k];
            fc = row[2 * na + k];
        } else {
            fa = A.vattr[(0 * na + k) * n + t];
            fb = A.vattr[(1 * na + k) * n + t];
            fc = A.vattr[(2 * na + k) * n + t];
        }
        return fmaf(b2, fc, fmaf(b1, fb, b0 * fa));
    };
    int k0 = 0;
    if (A.normalize3) {
        float n0 = interp(0), n1 = interp(1), n2 = interp(2);
        const float len2 = fmaf(n0, n0, fmaf(n1, n1, n2 * n2));
        if (len2 > 0.0f) {
            const float inv = 1.0f / sqrtf(len2);
            n0 *= inv;
            n1 *= inv;
            n2 *= inv;
        }
        A.attr[o] = n0;
        A.attr[plane + o] = n1;
        A.attr[2 * plane + o] = n2;
        k0 = 3;
    }
    for (int k = k0; k < A.nattr; ++k) A.attr[k * plane + o] = interp(k);
}

template <bool kPacked>
__global__ __launch_bounds__(256) void k_resolve(ResolveArgs A) {
    const int w = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    const int64_t tile = xcd_remap(blockIdx.x, gridDim.x) * 4 + w;
    if (tile >= A.ntiles) return;
    resolve_tile<kPacked>(A, tile, threadIdx.x & 63);
}

// 64 triangles per 256-thread workgroup, transposed through LDS: the
// [9][T] and [3][K][T] arrays are read along T and the rows written
// contiguously, so both sides stay coalesced.
constexpr int kPackTris = 64;

__global__ __launch_bounds__(256) void k_resolve_pack(const float* __restrict__ xyz, const float* __restrict__ vattr,
                                                      int64_t n, int32_t nattr, int32_t stride,
                                                      float* __restrict__ packed) {
    extern __shared__ float rows[];  // kPackTris x stride
    const int64_t t0 = int64_t(blockIdx.x) * kPackTris;
    const int nt = int(min(int64_t(kPackTris), n - t0));
    const int nq = 9 + 3 * nattr;
    for (int i = threadIdx.x; i < stride * kPackTris; i += 256) {
        const int q = i / kPackTris, tl = i % kPackTris;
        float v = 0.0f;
        if (tl < nt && q < nq) v = q < 9 ? xyz[int64_t(q) * n + t0 + tl] : vattr[int64_t(q - 9) * n + t0 + tl];
        rows[tl * stride + q] = v;
    }
    __syncthreads();
    float* out = packed + t0 * stride;
    for (int i = threadIdx.x; i < nt * stride; i += 256) out[i] = rows[i];
}

hipError_t launch_resolve_pack(const float* xyz, const float* vattr, int64_t n, int32_t nattr, void* packed,
                               hipStream_t st) {
    const int32_t stride = resolve_stride(nattr);
    if (n > 0)
        hipLaunchKernelGGL(k_resolve_pack, dim3(unsigned((n + kPackTris - 1) / kPackTris)), dim3(256),
                           size_t(kPackTris) * stride * 4, st, xyz, vattr, n, nattr, stride,
                           reinterpret_cast<float*>(packed));
    return hipGetLastError();
}

// packed (optional): rows from vsr_resolve_pack; then xyz and vattr are not read.
hipError_t launch_resolve(const void* map, int32_t W, int32_t H, int32_t fmt, const Rot& R, const float* xyz,
                          int64_t ntri, const uint32_t* tri_id, const float* vattr, int32_t nattr, bool normalize3,
                          float* bary, float* attr, hipStream_t st, const void* packed = nullptr) {
    const MapLayout ML = map_layout(W, H, fmt);
    ResolveArgs A;
    A.map = map;
    A.ntiles = ML.ntiles;
    A.fmt = fmt;
    A.W = W;
    A.H = H;
    A.ntx = ML.ntx;
    A.rot = R;
    A.xyz = xyz;
    A.ntri = ntri;
    A.tri_id = tri_id;
    A.vattr = vattr;
    A.nattr = nattr;
    A.normalize3 = normalize3 ? 1 : 0;
    A.bary = bary;
    A.attr = attr;
    A.packed = reinterpret_cast<const float*>(packed);
    A.stride = resolve_stride(nattr);
    A.pad_ = 0;
    if (packed)
        hipLaunchKernelGGL(k_resolve<true>, dim3(unsigned((ML.ntiles + 3) / 4)), dim3(256), 0, st, A);
    else
        hipLaunchKernelGGL(k_resolve<false>, dim3(unsigned((ML.ntiles + 3) / 4)), dim3(256), 0, st, A);
    return hipGetLastError();
}

}  // namespace vsr
