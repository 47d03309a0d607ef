// Fused, depth-sliced binning + rasterization (vsr_render, vsr_submit).
//
// One 256-thread workgroup renders a 16x16 super-tile (wave w: tile w).  The
// triangles are visited in groups of their nearest-first depth slices
// (ranks below n/64, n/16, n/4, n): for each group the candidates are
// gathered into the four tiles' LDS lists, each list is ordered by depth
// bucket and rasterized with the bucket early exit, and a tile is finished
// as soon as every one of its pixels holds a depth below the lower bound of
// the next group.  Far geometry behind a covered tile is then never even
// gathered.  A list that fills up is rasterized on the spot (flush) and
// emptied, so any depth complexity fits in LDS.
//
// Every path computes the exact minimum of the (depth, id) keys over the
// covering triangles — the exits only skip triangles that cannot win — so
// the images are bit-identical to vsr_bin + vsr_raster.
#pragma once
#include "raster.hpp"

namespace vsr {

constexpr int kFusedCap = 1024;                // LDS list entries per tile
constexpr int kFusedSteps = kSlices;  // one depth slice per step
constexpr uint32_t kFlushAt = kFusedCap - 256;  // a chunk adds <= 256 per tile

struct FusedArgs {
    const void* map;
    int64_t ntiles;
    int32_t fmt, W, H, ntx, nty, pad;
    const void* setup;
    int64_t n;
    uint32_t* scratch;  // kFusedCap ranks per tile (bucket-ordered lists)
    uint32_t* tri_id;
    float* depth;
    Rot rot;            // camera -> world

    __device__ inline void globalize() {
        map = to_global(map);
        setup = to_global(setup);
        scratch = to_global(scratch);
        tri_id = to_global(tri_id);
        depth = to_global(depth);
    }
};

__device__ inline void fused_super(const FusedArgs& A0, int64_t sidx) {
    FusedArgs A = A0;
    A.globalize();
    __shared__ uint32_t lists[kSupTiles][kFusedCap];
    __shared__ SuperShared sh;
    __shared__ float4 stage[kSupTiles][64];
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    int64_t tile;
    int tx, ty;
    const bool present = super_tile_of(sidx, w, A.ntx, A.nty, tile, tx, ty);
    super_setup(sh, map_caps(A.map, A.ntiles, A.fmt), map_sups(A.map, A.ntiles, A.fmt), A.rot,
                scene_view(A.setup, A.n).face_count, present, tile, sidx);
    const SceneView S = scene_view(A.setup, A.n);

    const int i = tx * kTile + (lane & (kTile - 1)), j = ty * kTile + (lane >> 3);
    const bool inside = present && i < A.W && j < A.H;
    float3 g = f3(0.f, 0.f, 0.f);
    if (present) g = load_dir(A.map, A.fmt, A.ntiles, tile, lane, A.rot);
    const bool has_dir = inside && (g.x != 0.0f || g.y != 0.0f || g.z != 0.0f);
    uint64_t best = kKeyEmpty;
    bool done = !present || sh.cap[w][1].z == kCapEmpty || A.n == 0;
    if (lane == 0) sh.flag[w] = done ? 1u : 0u;
    __syncthreads();

    unsigned long long n_tri = 0, n_cov = 0;  // unused counters of raster_list
    float4 tc0[kSupTiles], tc1[kSupTiles];
#pragma unroll
    for (int q = 0; q < kSupTiles; ++q) {
        tc0[q] = sh.cap[q][0];
        tc1[q] = sh.cap[q][1];
    }
    float4* stg = stage[w];
    uint32_t* my = lists[w];
    uint32_t* scr = A.scratch + (present ? tile : 0) * kFusedCap;
    const int shift = bucket_shift(A.n);

    // slice groups visited in turn
    for (int step = 0; step < kFusedSteps; ++step) {
        const int s0 = step, s1 = step + 1;
        uint32_t live = 0;
#pragma unroll
        for (int q = 0; q < kSupTiles; ++q)
            if (sh.flag[q] == 0u) live |= 1u << q;
        if (live == 0) break;
        auto append = [&](uint32_t mask, uint32_t rank) {
#pragma unroll
            for (int q = 0; q < kSupTiles; ++q) {
                if (mask & (1u << q)) {
                    uint32_t pos = atomicAdd(&sh.cnt[q], 1u);
                    lists[q][pos] = rank;
                }
            }
        };
        auto chunk_end = [&]() {
            __syncthreads();
            const uint32_t c = sh.cnt[w];
            if (c > kFlushAt) {
                if (!done) raster_list<false>(my, c, S.rec, g, has_dir, best, stg, false, n_tri, n_cov);
                if (lane == 0) sh.cnt[w] = 0;
            }
            __syncthreads();
        };
        auto visit = [&](bool valid, float4 a, float ch_t, float3 n0, float3 n1, float3 n2, uint32_t rank) {
            uint32_t mask = 0;
            if (valid) {
#pragma unroll
                for (int q = 0; q < kSupTiles; ++q)
                    if ((live >> q) & 1u)
                        if (sub_may_see(tc0[q], tc1[q], a, ch_t, n0, n1, n2)) mask |= 1u << q;
            }
            if (mask) append(mask, rank);
        };
        gather_slices(sh, S, s0, s1, [&](const uint32_t* chunk, uint32_t n) {
            const bool valid = uint32_t(threadIdx.x) < n;
            visit_record(S, valid, valid ? chunk[threadIdx.x] : 0u, visit);
        }, chunk_end);
        const uint32_t c = sh.cnt[w];
        if (!done && c > 0) {
            bucket_sort_wave(my, c, sh.bk[w], shift, scr);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            raster_list<false>(scr, c, S.rec, g, has_dir, best, stg, true, n_tri, n_cov);
        }
        if (!done) {
            // every later triangle has a depth lower bound >= that of the
            // first rank of the next group, floored to its sort key
            const int64_t nb = slice_begin(A.n, s1);
            if (nb < A.n) {
                float next_lb = depth_key_floor(S.rec[4 * nb + 3].y);
                uint32_t worst = wave_max_u32_dpp(has_dir ? uint32_t(best >> 32) : 0u);
                if (next_lb > __uint_as_float(worst)) done = true;
            }
        }
        if (lane == 0) {
            sh.flag[w] = done ? 1u : 0u;
            sh.cnt[w] = 0;
        }
        __syncthreads();
    }
    if (inside) {
        int64_t o = int64_t(j) * A.W + i;
        A.tri_id[o] = uint32_t(best & 0xFFFFFFFFull);
        A.depth[o] = __uint_as_float(uint32_t(best >> 32));
    }
}

__global__ __launch_bounds__(256) void k_fused(FusedArgs A) {
    const int64_t nsx = (A.ntx + 1) / 2;  // super-tiles per row
    fused_super(A, band_remap(blockIdx.x, gridDim.x, max(int64_t(1), nsx * kBandPx / (2 * kTile))));
}

inline int64_t fused_scratch_bytes(int32_t W, int32_t H) {
    return align256(map_layout(W, H, VSR_MAP_F32).ntiles * int64_t(kFusedCap) * 4);
}

hipError_t launch_fused(const void* map, int32_t W, int32_t H, int32_t fmt, const Rot& R, const void* setup, int64_t n,
                        void* scratch, uint32_t* tri_id, float* depth, hipStream_t st) {
    MapLayout ML = map_layout(W, H, fmt);
    FusedArgs A;
    A.map = map;
    A.ntiles = ML.ntiles;
    A.fmt = fmt;
    A.W = W;
    A.H = H;
    A.ntx = ML.ntx;
    A.nty = ML.nty;
    A.pad = 0;
    A.setup = setup;
    A.n = n;
    A.scratch = reinterpret_cast<uint32_t*>(scratch);
    A.tri_id = tri_id;
    A.depth = depth;
    A.rot = R;
    hipLaunchKernelGGL(k_fused, dim3(unsigned(bin_grid(ML.ntx, ML.nty))), dim3(256), 0, st, A);
    return hipGetLastError();
}

}  // namespace vsr
