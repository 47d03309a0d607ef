// Conservative binning (vsr_bin): per 8x8 tile, the triangles that may
// cover one of its pixels, in depth-bucket order.
//
// One 256-thread workgroup per 16x16 super-tile (2x2 tiles; wave w owns tile
// w): the super-tile cap is gathered once per depth slice (gather.hpp),
// survivors are appended to the four tiles' LDS lists with LDS atomics, and
// each wave writes its list with a counting sort by depth bucket.
#pragma once
#include "gather.hpp"

namespace vsr {

struct BinArgs {
    const void* map;
    int64_t ntiles;
    int32_t fmt, depth, lds_cap, all;
    int32_t ntx, nty;
    const void* setup;
    int64_t n;
    void* bins;
    uint32_t* status;  // overflowed-tile counter
    Rot rot;           // camera -> world
};

__device__ inline void bin_super(const BinArgs& A, int64_t sidx) {
    extern __shared__ uint32_t lists[];  // kSupTiles x lds_cap
    __shared__ SuperShared sh;
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    int64_t tile;
    int tx, ty;
    const bool present = super_tile_of(sidx, w, A.ntx, A.nty, tile, tx, ty);
    super_setup(sh, map_caps(A.map, A.ntiles, A.fmt), map_sups(A.map, A.ntiles, A.fmt), A.rot,
                scene_view(A.setup, A.n).face_count, present, tile, sidx);
    const bool any = sh.sup[1].z != 0.0f;
    const SceneView S = scene_view(A.setup, A.n);
    const uint32_t lcap = uint32_t(A.lds_cap);
    uint32_t live_mask = 0;
#pragma unroll
    for (int q = 0; q < kSupTiles; ++q)
        if (sh.cap[q][1].z != kCapEmpty) live_mask |= 1u << q;

    auto append = [&](uint32_t mask, uint32_t rank) {
#pragma unroll
        for (int q = 0; q < kSupTiles; ++q) {
            if (mask & (1u << q)) {
                uint32_t pos = atomicAdd(&sh.cnt[q], 1u);
                if (pos < lcap) lists[q * lcap + pos] = rank;
            }
        }
    };
    if (any && A.all) {
        for (int64_t k0 = 0; k0 < A.n; k0 += 256) {
            int64_t r = k0 + tid;
            if (r < A.n && S.cap[2 * r + 1].z != kCapEmpty) append(live_mask, uint32_t(r));
        }
    } else if (any) {
        gather_slices(sh, S, 0, kSlices, live_mask, append, [] {});
    }
    __syncthreads();

    const uint32_t cnt = sh.cnt[w];
    const bool keep = present && cnt <= uint32_t(A.depth);
    char* bb = reinterpret_cast<char*>(A.bins);
    if (keep) {
        uint32_t* out = reinterpret_cast<uint32_t*>(bb + 256 + align256(A.ntiles * 4)) + tile * A.depth;
        bucket_sort_wave(lists + w * lcap, cnt, sh.bk[w], bucket_shift(A.n), out);
    }
    if (present && lane == 0) {
        reinterpret_cast<uint32_t*>(bb + 256)[tile] = cnt;
        if (!keep) atomicAdd(A.status, 1u);
    }
}

__global__ __launch_bounds__(256) void k_bin(BinArgs A) { bin_super(A, xcd_remap(blockIdx.x, gridDim.x)); }

__global__ __launch_bounds__(64) void k_zero_u32(uint32_t* p, int64_t n) {
    int64_t i = int64_t(blockIdx.x) * 64 + threadIdx.x;
    if (i < n) p[i] = 0u;
}

inline int32_t bin_lds_cap(int32_t depth) {
    int32_t c = 64;
    while (c < depth) c <<= 1;
    return c;
}

inline int64_t bin_grid(int32_t ntx, int32_t nty) { return int64_t((ntx + 1) / 2) * ((nty + 1) / 2); }

hipError_t launch_bin(const void* map, int32_t W, int32_t H, int32_t fmt, const Rot& R, const void* setup, int64_t n,
                      int32_t depth, bool all, void* bins, hipStream_t st) {
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
    A.rot = R;
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, reinterpret_cast<uint32_t*>(bins), int64_t(64));
    hipLaunchKernelGGL(k_bin, dim3(unsigned(bin_grid(ML.ntx, ML.nty))), dim3(256),
                       size_t(kSupTiles) * A.lds_cap * 4, st, A);
    return hipGetLastError();
}

}  // namespace vsr
