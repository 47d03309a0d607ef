// Batched views: one launch per stage for any number of jobs — all maps,
// then either the binner over all jobs' 16x16 super-tiles and the
// rasterizer over all their 8x8 tiles (VSR_SUBMIT_BINNED), or the fused
// depth-sliced bin + raster over all super-tiles (VSR_SUBMIT_FUSED).
//
// Maps are camera-frame, so jobs whose lens (size, angle of view and
// effective k, l, s, Omega) is the same share one map, built once per
// submit; every job applies its own rotation.
//
// The job table lives in the workspace; it is written by a small kernel whose
// arguments carry the descriptors (no host-memory copy, so a caller may
// capture the whole submit in a HIP graph).  Each kernel maps its global
// tile (or super-tile) index to (job, local index), by one division when all
// jobs share one tile grid and otherwise with a uniform binary search over
// the jobs' offsets, and runs the per-tile device function of the
// single-view path, so a batched job's images are bit-identical to
// rendering that view alone.

#pragma once
#include <algorithm>
#include <array>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "fused.hpp"
#include "map.hpp"

namespace vsr {

int make_map_params(const vsr_view* v, int32_t fmt, uint32_t flags, MapParams* P, vsr_view* eff);

struct JobDesc {
    MapParams P;
    void* map;
    void* bins;
    const void* setup;
    int64_t ntri;
    uint32_t* tri_id;
    float* depth;
    int64_t tile_off;  // first global tile of this job
    int64_t ntiles;
    int64_t stile_off;  // first global super-tile (binning) of this job
    int64_t msup_off;   // first global map super-tile of this job's map (if it builds it)
    int64_t mblk_off;   // first global map block of this job's map (if it builds it)
    int64_t blk_off;    // first global 32x32 block (binning) of this job
    int32_t ntx, nty;
    int32_t map_owner;  // 1: this job builds the map it uses
    int32_t pad;
};

constexpr int kJobChunk = 8;
struct JobChunk {
    JobDesc d[kJobChunk];
    int32_t first, count;
};

__global__ void k_write_jobs(JobChunk c, JobDesc* table) {
    int q = threadIdx.x;
    if (q < c.count) table[c.first + q] = c.d[q];
}

// XCDs of the chip: workgroup b of a launch runs on XCD b mod kXcds.  The
// persistent rasterizers keep one work counter per XCD, 64 bytes apart.
constexpr int kXcds = 8;

// Workspace: 256-byte status header (word 0: overflowed tiles), the work
// counters, the job table, then the jobs' maps and bins.
struct WsLayout {
    int64_t ctr_off, table_off, data_off, bytes;
};

static WsLayout ws_layout(int32_t njobs) {
    WsLayout w;
    w.ctr_off = 256;
    w.table_off = w.ctr_off + int64_t(kXcds) * 64;
    w.data_off = w.table_off + align256(int64_t(njobs) * int64_t(sizeof(JobDesc)));
    w.bytes = w.data_off;
    return w;
}

inline int64_t job_scratch_bytes(int32_t W, int32_t H, int32_t mode, int32_t depth) {
    return mode == VSR_SUBMIT_FUSED ? fused_scratch_bytes(W, H) : bin_layout(W, H, depth).bytes;
}

int64_t submit_bytes(const vsr_job* jobs, int32_t njobs, int32_t fmt, int32_t mode, int32_t depth) {
    int64_t b = ws_layout(njobs).bytes;
    for (int32_t q = 0; q < njobs; ++q) {
        b += map_layout(jobs[q].view.width, jobs[q].view.height, fmt).bytes;
        b += job_scratch_bytes(jobs[q].view.width, jobs[q].view.height, mode, depth);
    }
    return b;
}

// Last job whose range offset (member Off) is <= t.  Jobs with empty
// ranges share the next job's offset and are never returned for t < total.
template <int64_t JobDesc::*Off>
__device__ inline int find_off(const JobDesc* __restrict__ T, int njobs, int64_t t) {
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (T[mid].*Off <= t)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Per-job range sizes when every job has the same tile grid (0 otherwise):
// then a global index maps to its job by one division instead of a binary
// search over the table, whose dependent loads open every workgroup.
struct JobGrid {
    int64_t tiles, stiles, blks;
};

template <int64_t JobDesc::*Off>
__device__ inline int job_of(const JobDesc* __restrict__ T, int njobs, int64_t per_job, int64_t t) {
    if (per_job > 0) return int(t / per_job);
    return find_off<Off>(T, njobs, t);
}

__global__ __launch_bounds__(256) void k_submit_bin_block(const JobDesc* __restrict__ T, int njobs, int32_t fmt,
                                                          int32_t depth, int32_t lds_cap, uint32_t* status, JobGrid G) {
    int64_t t = xcd_remap(blockIdx.x, gridDim.x);
    int jb = job_of<&JobDesc::blk_off>(T, njobs, G.blks, t);
    const JobDesc& J = T[jb];
    BinArgs A;
    A.map = J.map;
    A.ntiles = J.ntiles;
    A.fmt = fmt;
    A.depth = depth;
    A.lds_cap = lds_cap;
    A.all = 0;
    A.ntx = J.ntx;
    A.nty = J.nty;
    A.tile16 = 0;
    A.pad = 0;
    A.setup = J.setup;
    A.n = J.ntri;
    A.bins = J.bins;
    A.status = status;
    A.rot = rot_of(J.P.rot);
    bin_block(A, t - J.blk_off);
}

__global__ __launch_bounds__(256) VSR_BLOCK16_WAVES void k_submit_bin_block16(const JobDesc* __restrict__ T, int njobs, int32_t fmt,
                                                      int32_t depth, int32_t lds_cap, uint32_t* status, JobGrid G) {
    int64_t t = xcd_remap(blockIdx.x, gridDim.x);
    int jb = job_of<&JobDesc::blk_off>(T, njobs, G.blks, t);
    const JobDesc& J = T[jb];
    BinArgs A;
    A.map = J.map;
    A.ntiles = J.ntiles;
    A.fmt = fmt;
    A.depth = depth;
    A.lds_cap = lds_cap;
    A.all = 0;
    A.ntx = J.ntx;
    A.nty = J.nty;
    A.tile16 = 1;
    A.pad = 0;
    A.setup = J.setup;
    A.n = J.ntri;
    A.bins = J.bins;
    A.status = status;
    A.rot = rot_of(J.P.rot);
    bin_block16(A, t - J.blk_off);
}

__global__ __launch_bounds__(256) void k_submit_bin16(const JobDesc* __restrict__ T, int njobs, int32_t fmt,
                                                      int32_t depth, int32_t lds_cap, uint32_t* status, JobGrid G) {
    int64_t t = xcd_remap(blockIdx.x, gridDim.x);
    int jb = job_of<&JobDesc::stile_off>(T, njobs, G.stiles, t);
    const JobDesc& J = T[jb];
    BinArgs A;
    A.map = J.map;
    A.ntiles = J.ntiles;
    A.fmt = fmt;
    A.depth = depth;
    A.lds_cap = lds_cap;
    A.all = 0;
    A.ntx = J.ntx;
    A.nty = J.nty;
    A.tile16 = 1;
    A.pad = 0;
    A.setup = J.setup;
    A.n = J.ntri;
    A.bins = J.bins;
    A.status = status;
    A.rot = rot_of(J.P.rot);
    bin_super16(A, t - J.stile_off);
}

__global__ __launch_bounds__(64) void k_submit_block_caps(const JobDesc* __restrict__ T, int njobs, int32_t fmt,
                                                          int64_t total) {
    const int64_t t = int64_t(blockIdx.x) * 64 + threadIdx.x;
    if (t >= total) return;
    const JobDesc& J = T[find_off<&JobDesc::mblk_off>(T, njobs, t)];
    block_cap(J.map, J.ntiles, fmt, J.ntx, J.nty, t - J.mblk_off);
}

__global__ __launch_bounds__(256) void k_submit_bin(const JobDesc* __restrict__ T, int njobs, int32_t fmt,
                                                    int32_t depth, int32_t lds_cap, uint32_t* status, JobGrid G) {
    int64_t t = xcd_remap(blockIdx.x, gridDim.x);
    int jb = job_of<&JobDesc::stile_off>(T, njobs, G.stiles, t);
    const JobDesc& J = T[jb];
    BinArgs A;
    A.map = J.map;
    A.ntiles = J.ntiles;
    A.fmt = fmt;
    A.depth = depth;
    A.lds_cap = lds_cap;
    A.all = 0;
    A.ntx = J.ntx;
    A.nty = J.nty;
    A.tile16 = 0;
    A.pad = 0;
    A.setup = J.setup;
    A.n = J.ntri;
    A.bins = J.bins;
    A.status = status;
    A.rot = rot_of(J.P.rot);
    bin_super(A, t - J.stile_off);
}

__global__ __launch_bounds__(256) void k_submit_raster(const JobDesc* __restrict__ T, int njobs, int32_t fmt,
                                                       int32_t depth, int64_t total, JobGrid G) {
    int w = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    int64_t t = xcd_remap(blockIdx.x, gridDim.x) * 4 + w;
    if (t >= total) return;
    int jb = job_of<&JobDesc::tile_off>(T, njobs, G.tiles, t);
    const JobDesc& J = T[jb];
    RasterArgs A;
    A.map = J.map;
    A.ntiles = J.ntiles;
    A.fmt = fmt;
    A.depth = depth;
    A.W = J.P.W;
    A.H = J.P.H;
    A.ntx = J.P.ntx;
    A.nty = J.P.nty;
    A.setup = J.setup;
    A.n = J.ntri;
    A.bins = J.bins;
    A.tri_id = J.tri_id;
    A.out_depth = J.depth;
    A.stats = nullptr;
    A.no_early_exit = 0;
    A.rot = rot_of(J.P.rot);
    raster_tile<false>(A, t - J.tile_off, threadIdx.x & 63);
}

// 16x16 bin tiles: kStripTiles super-tiles of the jobs' concatenated range
// per workgroup, each wave on kStripTiles of a super-tile's 8x8 tiles
__global__ __launch_bounds__(256) void k_submit_raster16(const JobDesc* __restrict__ T, int njobs, int32_t fmt,
                                                         int32_t depth, int64_t total, JobGrid G) {
    constexpr int kWps = 4 / kStripTiles;
    __shared__ float4 s_stage16[4][256];
    const int w = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    const int64_t t = kStripTiles * xcd_remap(blockIdx.x, gridDim.x) + w / kWps;
    if (t >= total) return;
    const int jb = job_of<&JobDesc::stile_off>(T, njobs, G.stiles, t);
    const JobDesc& J = T[jb];
    RasterArgs A;
    A.map = J.map;
    A.ntiles = J.ntiles;
    A.fmt = fmt;
    A.depth = depth;
    A.W = J.P.W;
    A.H = J.P.H;
    A.ntx = J.P.ntx;
    A.nty = J.P.nty;
    A.setup = J.setup;
    A.n = J.ntri;
    A.bins = J.bins;
    A.tri_id = J.tri_id;
    A.out_depth = J.depth;
    A.stats = nullptr;
    A.no_early_exit = 0;
    A.rot = rot_of(J.P.rot);
    raster_multi16<false, kStripTiles>(A, t - J.stile_off, w % kWps, s_stage16[w]);
}

// Persistent rasterizers (VSR_SUBMIT_PERSISTENT): a grid of about as many
// workgroups as are resident at once; each wave takes runs of kWorkChunk
// work items (an 8x8 tile; with 16x16 lists a (super-tile, quadrant) pair,
// the four quadrants of a super-tile being consecutive items) from work
// counters until none are left.  The items are split into kXcds contiguous
// ranges with a counter each; range r belongs to XCD r, and a wave visits
// every range once, its XCD's first, so neighbouring tiles, which share
// triangles, meet in one L2.  Within a range the items come in increasing order, so a wave finds
// each item's job by walking forward from the last one (a binary search
// only after a move).  The counters sit in the workspace (zeroed by the
// submit); the per-tile work is the grid kernels', so the images are the
// same.  Measured slower than the grid kernels on 64 1080p views (the
// vector memory counter covers loads and stores alike, so the first load
// wait of each tile also waits for the previous tile's output stores, and
// the loop needs more registers); kept as a measured alternative.
constexpr uint32_t kShapePersistent = 0x10000u;
constexpr int kPersistentWgPerCu = 8;
constexpr uint32_t kWorkChunk = 16;

// Compute units of the current device (cached per device).
static int device_cus() {
    static std::mutex mu;
    static std::map<int, int> cus;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    std::lock_guard<std::mutex> lock(mu);
    auto it = cus.find(dev);
    if (it != cus.end()) return it->second;
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n < 1) n = 256;
    cus.emplace(dev, n);
    return n;
}

template <int64_t JobDesc::*Off>
__device__ inline int advance_job(const JobDesc* __restrict__ T, int njobs, int jb, int64_t t) {
    if (jb < 0 || t < T[jb].*Off) return find_off<Off>(T, njobs, t);
    while (jb + 1 < njobs && T[jb + 1].*Off <= t) ++jb;
    return jb;
}

// Next run of up to kWorkChunk items [t, t_end) for the calling wave;
// false when it has found every range used up.  j counts the ranges it has
// left behind (its XCD's first, then the next XCD's, ...); jb is reset on a
// move.
__device__ inline bool next_items(uint32_t* __restrict__ ctr, int64_t items, int xcd, int& j, int& jb, int64_t& t,
                                  int64_t& t_end) {
    const int64_t per = (items + kXcds - 1) / kXcds;
    while (j < kXcds) {
        const int r = (xcd + j) % kXcds;
        uint32_t i = 0;
        if ((threadIdx.x & 63) == 0) i = atomicAdd(&ctr[16 * r], kWorkChunk);
        i = __builtin_amdgcn_readfirstlane(i);
        const int64_t end = min(int64_t(r + 1) * per, items);
        t = int64_t(r) * per + int64_t(i);
        if (int64_t(i) < per && t < end) {
            t_end = min(t + int64_t(kWorkChunk), end);
            return true;
        }
        ++j;
        jb = -1;
    }
    return false;
}

__device__ inline RasterArgs submit_raster_args(const JobDesc& J, int32_t fmt, int32_t depth) {
    RasterArgs A;
    A.map = J.map;
    A.ntiles = J.ntiles;
    A.fmt = fmt;
    A.depth = depth;
    A.W = J.P.W;
    A.H = J.P.H;
    A.ntx = J.P.ntx;
    A.nty = J.P.nty;
    A.setup = J.setup;
    A.n = J.ntri;
    A.bins = J.bins;
    A.tri_id = J.tri_id;
    A.out_depth = J.depth;
    A.stats = nullptr;
    A.no_early_exit = 0;
    A.rot = rot_of(J.P.rot);
    return A;
}

__global__ __launch_bounds__(256) void k_submit_raster_p(const JobDesc* __restrict__ T, int njobs, int32_t fmt,
                                                         int32_t depth, int64_t items, uint32_t* __restrict__ ctr) {
    const int xcd = int(blockIdx.x % kXcds);
    int j = 0, jb = -1;
    int64_t t0, t1;
    while (next_items(ctr, items, xcd, j, jb, t0, t1)) {
        for (int64_t t = t0; t < t1; ++t) {
            jb = advance_job<&JobDesc::tile_off>(T, njobs, jb, t);
            const JobDesc& J = T[jb];
            raster_tile<false>(submit_raster_args(J, fmt, depth), t - J.tile_off, threadIdx.x & 63);
        }
    }
}

__global__ __launch_bounds__(256) void k_submit_raster16_p(const JobDesc* __restrict__ T, int njobs, int32_t fmt,
                                                           int32_t depth, int64_t items, uint32_t* __restrict__ ctr) {
    __shared__ float4 s_stage[4][256];
    const int w = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    const int xcd = int(blockIdx.x % kXcds);
    int j = 0, jb = -1;
    int64_t t0, t1;
    while (next_items(ctr, items, xcd, j, jb, t0, t1)) {
        for (int64_t t = t0; t < t1; ++t) {
            const int64_t sidx = t >> 2;
            jb = advance_job<&JobDesc::stile_off>(T, njobs, jb, sidx);
            const JobDesc& J = T[jb];
            raster_quad16<false>(submit_raster_args(J, fmt, depth), sidx - J.stile_off, int(t & 3), s_stage[w]);
        }
    }
}

__global__ __launch_bounds__(256) void k_submit_fused(const JobDesc* __restrict__ T, int njobs, int32_t fmt, JobGrid G) {
    int64_t t = xcd_remap(blockIdx.x, gridDim.x);
    int jb = job_of<&JobDesc::stile_off>(T, njobs, G.stiles, t);
    const JobDesc& J = T[jb];
    FusedArgs A;
    A.map = J.map;
    A.ntiles = J.ntiles;
    A.fmt = fmt;
    A.W = J.P.W;
    A.H = J.P.H;
    A.ntx = J.ntx;
    A.nty = J.nty;
    A.pad = 0;
    A.setup = J.setup;
    A.n = J.ntri;
    A.scratch = reinterpret_cast<uint32_t*>(J.bins);
    A.tri_id = J.tri_id;
    A.depth = J.depth;
    A.rot = rot_of(J.P.rot);
    fused_super(A, t - J.stile_off);
}

// Map super-tiles of the jobs that own a map: job ranges [msup_off,
// msup_off + nsup) for owners, empty for sharers (whose offset equals the
// next job's, so the last job with msup_off <= t is always the owner of t).
__device__ inline int find_map_job(const JobDesc* __restrict__ T, int njobs, int64_t t) {
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (T[mid].msup_off <= t)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(256) void k_submit_map(const JobDesc* __restrict__ T, int njobs) {
    const int64_t t = blockIdx.x;
    const int jb = find_map_job(T, njobs, t);
    const JobDesc& J = T[jb];
    build_map_super(J.P, J.map, J.ntiles, t - J.msup_off);
}

// Job descriptors of a submit, in workspace order; returns the number of
// tiles, super-tiles and map super-tiles through the pointers.  With share_maps,
// jobs with the same lens use the first such job's map.
static void build_table(const vsr_job* jobs, int32_t njobs, int32_t fmt, int32_t mode, int32_t depth, void* ws,
                        bool share_maps, JobDesc* out, int64_t* n_tiles, int64_t* n_stiles, int64_t* n_mtiles,
                        int64_t* n_blks, int64_t* n_mblks) {
    WsLayout W = ws_layout(njobs);
    char* base = reinterpret_cast<char*>(ws);
    int64_t off = W.data_off, tiles = 0, stiles = 0, mtiles = 0, blks = 0, mblks = 0;
    std::map<std::array<uint32_t, 7>, int32_t> lens;
    auto bits = [](float f) {
        uint32_t u;
        memcpy(&u, &f, 4);
        return u;
    };
    for (int32_t q = 0; q < njobs; ++q) {
        JobDesc& D = out[q];
        vsr_view eff;
        make_map_params(&jobs[q].view, fmt, 0, &D.P, &eff);
        MapLayout ML = map_layout(D.P.W, D.P.H, fmt);
        const std::array<uint32_t, 7> key = {uint32_t(eff.width), uint32_t(eff.height), uint32_t(eff.aov),
                                             bits(eff.k), bits(eff.l), bits(eff.s), bits(eff.omega_deg)};
        auto it = share_maps ? lens.find(key) : lens.end();
        D.msup_off = mtiles;
        D.mblk_off = mblks;
        if (it != lens.end()) {
            D.map = out[it->second].map;
            D.map_owner = 0;
        } else {
            D.map = base + off;
            off += ML.bytes;
            D.map_owner = 1;
            mtiles += ML.nsup;
            mblks += ML.nblk;
            if (share_maps) lens.emplace(key, q);
        }
        D.pad = 0;
        D.bins = base + off;
        off += job_scratch_bytes(D.P.W, D.P.H, mode, depth);
        D.ntx = ML.ntx;
        D.nty = ML.nty;
        D.stile_off = stiles;
        stiles += bin_grid(ML.ntx, ML.nty);
        D.blk_off = blks;
        blks += ML.nblk;
        D.setup = jobs[q].setup;
        D.ntri = jobs[q].ntri;
        D.tri_id = jobs[q].tri_id;
        D.depth = jobs[q].depth;
        D.tile_off = tiles;
        D.ntiles = ML.ntiles;
        tiles += ML.ntiles;
    }
    *n_tiles = tiles;
    *n_stiles = stiles;
    *n_mtiles = mtiles;
    *n_blks = blks;
    *n_mblks = mblks;
}

int64_t submit_table_bytes(int32_t njobs) { return int64_t(njobs) * int64_t(sizeof(JobDesc)); }

// Host image of the job table that vsr_submit would write into `ws`.
void submit_table(const vsr_job* jobs, int32_t njobs, int32_t fmt, int32_t mode, int32_t depth, void* ws,
                  void* host) {
    int64_t t, s, m, b, mb;
    build_table(jobs, njobs, fmt, mode, depth, ws, false, reinterpret_cast<JobDesc*>(host), &t, &s, &m, &b, &mb);
}

int64_t submit_table_offset() { return ws_layout(1).table_off; }

// ev (optional): four events recorded on st before the maps, before the
// binner (or the fused kernel), before the rasterizer and after the last
// kernel, for timing the stages.
hipError_t launch_submit(const vsr_job* jobs, int32_t njobs, int32_t fmt, int32_t mode, int32_t depth, void* ws,
                         bool table_ready, uint32_t shape, hipStream_t st, hipEvent_t* ev = nullptr) {
    WsLayout W = ws_layout(njobs);
    char* base = reinterpret_cast<char*>(ws);
    JobDesc* table = reinterpret_cast<JobDesc*>(base + W.table_off);
    std::vector<JobDesc> host(njobs);
    int64_t tiles = 0, stiles = 0, mtiles = 0, blks = 0, mblks = 0;
    // a prewritten table (graph replays) never shares maps, so the grids
    // sized here fit any table written for jobs of the same sizes
    build_table(jobs, njobs, fmt, mode, depth, ws, !table_ready, host.data(), &tiles, &stiles, &mtiles, &blks,
                &mblks);
    JobGrid G = {0, 0, 0};
    bool same = true;
    for (int32_t q = 1; q < njobs; ++q) same = same && host[q].ntx == host[0].ntx && host[q].nty == host[0].nty;
    if (same) {
        G.tiles = host[0].ntiles;
        G.stiles = bin_grid(host[0].ntx, host[0].nty);
        G.blks = blks / njobs;
    }
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, reinterpret_cast<uint32_t*>(ws), int64_t(64));
    if (!table_ready) {
        // descriptors travel as kernel arguments: no host-memory copy
        for (int32_t first = 0; first < njobs; first += kJobChunk) {
            JobChunk chunk;
            chunk.first = first;
            chunk.count = std::min(kJobChunk, njobs - first);
            for (int q = 0; q < chunk.count; ++q) chunk.d[q] = host[first + q];
            hipLaunchKernelGGL(k_write_jobs, dim3(1), dim3(kJobChunk), 0, st, chunk, table);
        }
    }
    if (ev) (void)hipEventRecord(ev[0], st);
    if (mtiles > 0) hipLaunchKernelGGL(k_submit_map, dim3(unsigned(mtiles)), dim3(256), 0, st, table, njobs);
    if (mblks > 0)
        hipLaunchKernelGGL(k_submit_block_caps, dim3(unsigned((mblks + 63) / 64)), dim3(64), 0, st, table, njobs, fmt,
                           mblks);
    if (ev) (void)hipEventRecord(ev[1], st);
    if (mode == VSR_SUBMIT_FUSED) {
        hipLaunchKernelGGL(k_submit_fused, dim3(unsigned(stiles)), dim3(256), 0, st, table, njobs, fmt, G);
        if (ev) (void)hipEventRecord(ev[2], st);
    } else {
        int32_t cap = bin_lds_cap(depth);
        const bool t16 = (shape & VSR_BIN_TILE16) != 0;
        if (t16 && use_blocks(cap, blks, shape, true))
            hipLaunchKernelGGL(k_submit_bin_block16, dim3(unsigned(blks)), dim3(256), size_t(4) * cap * 4, st,
                               table, njobs, fmt, depth, cap, reinterpret_cast<uint32_t*>(ws), G);
        else if (t16)
            hipLaunchKernelGGL(k_submit_bin16, dim3(unsigned(stiles)), dim3(256), size_t(cap) * 4, st,
                               table, njobs, fmt, depth, cap, reinterpret_cast<uint32_t*>(ws), G);
        else if (use_blocks(cap, blks, shape))
            hipLaunchKernelGGL(k_submit_bin_block, dim3(unsigned(blks)), dim3(256), 0, st,
                               table, njobs, fmt, depth, cap, reinterpret_cast<uint32_t*>(ws), G);
        else
            hipLaunchKernelGGL(k_submit_bin, dim3(unsigned(stiles)), dim3(256), size_t(kSupTiles) * cap * 4, st,
                               table, njobs, fmt, depth, cap, reinterpret_cast<uint32_t*>(ws), G);
        if (ev) (void)hipEventRecord(ev[2], st);
        if (shape & kShapePersistent) {
            // as many workgroups as are resident at once, at most one wave
            // per item
            const int64_t items = t16 ? 4 * stiles : tiles;
            const int64_t wgs = std::min(int64_t(device_cus()) * kPersistentWgPerCu, (items + 3) / 4);
            uint32_t* ctr = reinterpret_cast<uint32_t*>(base + W.ctr_off);
            hipLaunchKernelGGL(k_zero_u32, dim3(unsigned(kXcds * 16 / 64)), dim3(64), 0, st, ctr,
                               int64_t(kXcds) * 16);
            if (t16)
                hipLaunchKernelGGL(k_submit_raster16_p, dim3(unsigned(wgs)), dim3(256), 0, st, table, njobs, fmt,
                                   depth, items, ctr);
            else
                hipLaunchKernelGGL(k_submit_raster_p, dim3(unsigned(wgs)), dim3(256), 0, st, table, njobs, fmt,
                                   depth, items, ctr);
        } else if (t16) {
            hipLaunchKernelGGL(k_submit_raster16, dim3(unsigned((stiles + kStripTiles - 1) / kStripTiles)), dim3(256),
                               0, st, table, njobs, fmt, depth, stiles, G);
        } else {
            hipLaunchKernelGGL(k_submit_raster, dim3(unsigned((tiles + 3) / 4)), dim3(256), 0, st, table, njobs, fmt,
                               depth, tiles, G);
        }
    }
    if (ev) (void)hipEventRecord(ev[3], st);
    return hipGetLastError();
}

}  // namespace vsr
