// C ABI of libvsr: argument checks, per-view constants, launches.
#include <math.h>
#include <stdio.h>
#include <string.h>

#pragma once
#include <stdarg.h>

#include "aa.hpp"
#include "bin.hpp"
#include "calib.hpp"
#include "fused.hpp"
#include "map.hpp"
#include "raster.hpp"
#include "resolve.hpp"
#include "setup.hpp"
#include "submit.hpp"
#include "wire.hpp"

using namespace vsr;

static thread_local char g_err[512] = "";

static int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
static int fail(int code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

static int hip_status(hipError_t e, const char* what) {
    if (e == hipSuccess) return VSR_OK;
    return fail(VSR_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

static bool aligned(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 255u) == 0; }

static const int32_t kMaxDim = 32768;
static const int32_t kMaxDepth = 2048;  // four lists of this many entries fit in LDS

// Section 2.1.1 limits, in double precision on float inputs.
static void limit_params(double& k, double& l, double& s, double& om) {
    k = k < -1.0 ? -1.0 : (k > 1.0 ? 1.0 : k);
    l = l < 0.0 ? 0.0 : (l > 1.0 ? 1.0 : l);
    s = s < 0.8 ? 0.8 : (s > 1.0 ? 1.0 : s);
    double om_max = (k > 0.0 ? 179.0 : 180.0) / fmax(fabs(k), 0.5);
    om = om < 1.0 ? 1.0 : (om > om_max ? om_max : om);
}

namespace vsr {
// Fills the per-view constants; returns VSR_OK or an error code.
int make_map_params(const vsr_view* v, int32_t fmt, uint32_t flags, MapParams* P, vsr_view* eff) {
    if (!v) return fail(VSR_E_ARG, "view is NULL");
    if (v->width < 1 || v->height < 1 || v->width > kMaxDim || v->height > kMaxDim)
        return fail(VSR_E_ARG, "view size %dx%d outside 1..%d", v->width, v->height, kMaxDim);
    if (v->aov < 0 || v->aov > 3) return fail(VSR_E_ARG, "unknown angle-of-view type %d", v->aov);
    if (fmt != VSR_MAP_F32 && fmt != VSR_MAP_OCT16) return fail(VSR_E_ARG, "unknown map format %d", fmt);
    double k = v->k, l = v->l, s = v->s, om = v->omega_deg;
    if (!(isfinite(k) && isfinite(l) && isfinite(s) && isfinite(om)))
        return fail(VSR_E_ARG, "non-finite view parameter");
    for (int q = 0; q < 9; ++q)
        if (!isfinite(v->rot[q])) return fail(VSR_E_ARG, "non-finite rotation");
    double k0 = k, l0 = l, s0 = s, om0 = om;
    limit_params(k, l, s, om);
    if ((flags & VSR_STRICT) && (k != k0 || l != l0 || s != s0 || om != om0))
        return fail(VSR_E_RANGE, "parameters (k=%g l=%g s=%g omega=%g) outside the limits", k0, l0, s0, om0);
    MapLayout L = map_layout(v->width, v->height, fmt);
    P->W = v->width;
    P->H = v->height;
    P->aov = v->aov;
    P->fmt = fmt;
    P->ntx = L.ntx;
    P->nty = L.nty;
    const double pi = 3.14159265358979323846;
    double half = 0.5 * om * pi / 180.0;
    P->kind = k > 0.0 ? 1 : (k < 0.0 ? -1 : 0);
    P->k = float(k);
    P->half = float(half);
    double kt = k > 0.0 ? tan(k * half) : (k < 0.0 ? sin(k * half) : 0.0);
    P->kt = float(kt);
    P->kt_lo = float(kt - double(P->kt));
    P->sig0 = float(k > 0.0 ? tan(k * half) / k : (k < 0.0 ? sin(k * half) / k : half));
    P->l = float(l);
    P->c = float(l * (1.0 - s) + s);
    double W = v->width, H = v->height;
    switch (v->aov) {
    case VSR_AOV_DIAGONAL:  // x = cx*a/sqrt(1+a^2) = (2i+1-W)/hypot(W,H)
        P->xmul = 1;
        P->xden = P->yden = float(sqrt(W * W + H * H));
        break;
    case VSR_AOV_VERTICAL:  // x = cx*a = (2i+1-W)/H
        P->xmul = 1;
        P->xden = P->yden = float(H);
        break;
    case VSR_AOV_HORIZONTAL_4X3:  // x = cx*a*3/4 = 3(2i+1-W)/(4H)
        P->xmul = 3;
        P->xden = P->yden = float(4.0 * H);
        break;
    default:  // horizontal: x = cx, y = cy/a = (2j+1-H)/W
        P->xmul = 1;
        P->xden = P->yden = float(W);
        break;
    }
    P->xden_lo = float(0.0);
    P->yden_lo = float(0.0);
    if (v->aov == VSR_AOV_DIAGONAL) {
        double hyp = sqrt(W * W + H * H);
        P->xden_lo = P->yden_lo = float(hyp - double(P->xden));
    }
    P->rxden = P->ryden = float(1.0 / (double(P->xden) + double(P->xden_lo)));
    P->rc = float(1.0 / (l * (1.0 - s) + s));
    for (int q = 0; q < 9; ++q) P->rot[q] = v->rot[q];
    P->lens = VSR_LENS_UNIVERSAL;
    P->lens_n = 1;
    P->distort = 0;
    P->fringe = 0.5f;
    for (int q = 0; q < 8; ++q) P->lp[q] = 0.0f;
    if (eff) {
        *eff = *v;
        eff->k = float(k);
        eff->l = float(l);
        eff->s = float(s);
        eff->omega_deg = float(om);
    }
    return VSR_OK;
}
// Generator constants of a vsr_lens (on top of make_map_params, whose
// Universal Perspective part the other generators ignore).
int make_lens_params(const vsr_lens* lens, MapParams* P) {
    if (!lens) return fail(VSR_E_ARG, "lens is NULL");
    for (int q = 0; q < 8; ++q)
        if (!isfinite(lens->p[q])) return fail(VSR_E_ARG, "non-finite lens parameter");
    const double pi = 3.14159265358979323846;
    const double W = P->W, H = P->H;
    P->lens = lens->type;
    switch (lens->type) {
    case VSR_LENS_UNIVERSAL: {
        bool any = false;
        for (int q = 0; q < 6; ++q) {
            P->lp[q] = lens->p[q];
            any = any || lens->p[q] != 0.0f;
        }
        P->distort = any ? 1 : 0;
        break;
    }
    case VSR_LENS_EQUIRECT:
    case VSR_LENS_CUBE:
        break;
    case VSR_LENS_SCREENS: {
        if (lens->n < 1 || lens->n > 64) return fail(VSR_E_ARG, "screen count %d outside 1..64", lens->n);
        double om = lens->p[0];
        if (!(om > 0.0 && om < 180.0)) return fail(VSR_E_ARG, "screen angle of view %g outside (0, 180)", om);
        P->lens_n = lens->n;
        P->lp[0] = float(1.0 / tan(0.5 * om * pi / 180.0));
        P->lp[1] = float(0.5 * om * pi / 180.0);
        break;
    }
    case VSR_LENS_VR: {
        double om = lens->p[0], d = lens->p[1], k1 = lens->p[2], k2 = lens->p[3];
        if (!(om > 0.0 && om < 180.0)) return fail(VSR_E_ARG, "vertical angle of view %g outside (0, 180)", om);
        if (!(fabs(1.0 + k1 + k2) > 1e-6)) return fail(VSR_E_ARG, "1 + k1 + k2 is zero");
        P->lp[0] = float(1.0 / tan(0.5 * om * pi / 180.0));
        P->lp[1] = float(1.0 - 2.0 * d);
        P->lp[2] = float(k1);
        P->lp[3] = float(k2);
        P->lp[4] = float(1.0 / (1.0 + k1 + k2));
        P->lp[5] = float(0.5 * W / H);
        break;
    }
    case VSR_LENS_PANORAMA: {
        double om = lens->p[0];
        if (!(om > 0.0 && om <= 360.0)) return fail(VSR_E_ARG, "panorama angle of view %g outside (0, 360]", om);
        P->lp[0] = float(om * pi / 180.0 / (2.0 * W));
        break;
    }
    case VSR_LENS_DOME: {
        double comp = lens->p[0], tilt = lens->p[1] * pi / 180.0, off = lens->p[2];
        if (!(comp >= -89.0 && comp <= 90.0)) return fail(VSR_E_ARG, "dome compression %g outside [-89, 90]", comp);
        if (!(off > -1.0 && off < 1.0)) return fail(VSR_E_ARG, "dome offset %g outside (-1, 1)", off);
        P->lp[0] = float((comp + 90.0) * pi / 180.0);
        P->lp[1] = float(sin(tilt));
        P->lp[2] = float(cos(tilt));
        P->lp[3] = float(off);
        break;
    }
    default:
        return fail(VSR_E_ARG, "unknown lens type %d", lens->type);
    }
    return VSR_OK;
}
}  // namespace vsr

extern "C" {

int64_t vsr_map_bytes(int32_t width, int32_t height, int32_t fmt) {
    if (width < 1 || height < 1 || width > kMaxDim || height > kMaxDim) return VSR_E_ARG;
    if (fmt != VSR_MAP_F32 && fmt != VSR_MAP_OCT16) return VSR_E_ARG;
    return map_layout(width, height, fmt).bytes;
}

int64_t vsr_setup_bytes(int64_t ntri) {
    if (ntri < 0 || ntri > (int64_t(1) << 31)) return VSR_E_ARG;
    return setup_layout(ntri).bytes;
}

int64_t vsr_bin_bytes(int32_t width, int32_t height, int32_t bin_depth) {
    if (width < 1 || height < 1 || width > kMaxDim || height > kMaxDim) return VSR_E_ARG;
    if (bin_depth < 1 || bin_depth > kMaxDepth) return VSR_E_ARG;
    return bin_layout(width, height, bin_depth).bytes;
}

int vsr_build_map(const vsr_view* v, int32_t fmt, uint32_t flags, void* map, int64_t map_bytes, vsr_view* v_eff,
                  void* stream) {
    MapParams P;
    int rc = make_map_params(v, fmt, flags, &P, v_eff);
    if (rc != VSR_OK) return rc;
    if (!map || !aligned(map)) return fail(VSR_E_ARG, "map buffer NULL or not 256-byte aligned");
    if ((flags & ~(VSR_STRICT | VSR_MAP_AA | VSR_MAP_AA_LINES)) != 0) return fail(VSR_E_ARG, "unknown flags 0x%x", flags);
    const bool aa = (flags & (VSR_MAP_AA | VSR_MAP_AA_LINES)) != 0;
    if (flags & VSR_MAP_AA_LINES) P.fringe = 1.25f;
    int64_t need = aa ? aa_map_bytes(v->width, v->height, fmt) : map_layout(v->width, v->height, fmt).bytes;
    if (map_bytes < need) return fail(VSR_E_SPACE, "map buffer %lld < %lld bytes", (long long)map_bytes, (long long)need);
    return hip_status(launch_build_map(P, map, aa, hipStream_t(stream)), "vsr_build_map");
}

int vsr_build_map_lens(const vsr_view* v, const vsr_lens* lens, int32_t fmt, uint32_t flags, void* map,
                       int64_t map_bytes, vsr_view* v_eff, void* stream) {
    MapParams P;
    // the Universal Perspective parameters are limited (and checked under
    // VSR_STRICT) only when that generator is used
    const uint32_t base_flags = (lens && lens->type != VSR_LENS_UNIVERSAL) ? (flags & ~VSR_STRICT) : flags;
    int rc = make_map_params(v, fmt, base_flags, &P, v_eff);
    if (rc != VSR_OK) return rc;
    rc = make_lens_params(lens, &P);
    if (rc != VSR_OK) return rc;
    if (!map || !aligned(map)) return fail(VSR_E_ARG, "map buffer NULL or not 256-byte aligned");
    if ((flags & ~(VSR_STRICT | VSR_MAP_AA | VSR_MAP_AA_LINES)) != 0) return fail(VSR_E_ARG, "unknown flags 0x%x", flags);
    const bool aa = (flags & (VSR_MAP_AA | VSR_MAP_AA_LINES)) != 0;
    if (flags & VSR_MAP_AA_LINES) P.fringe = 1.25f;
    int64_t need = aa ? aa_map_bytes(v->width, v->height, fmt) : map_layout(v->width, v->height, fmt).bytes;
    if (map_bytes < need) return fail(VSR_E_SPACE, "map buffer %lld < %lld bytes", (long long)map_bytes, (long long)need);
    return hip_status(launch_build_map(P, map, aa, hipStream_t(stream)), "vsr_build_map_lens");
}

int64_t vsr_aa_map_bytes(int32_t width, int32_t height, int32_t fmt) {
    if (width < 1 || height < 1 || width > kMaxDim || height > kMaxDim) return VSR_E_ARG;
    if (fmt != VSR_MAP_F32 && fmt != VSR_MAP_OCT16) return VSR_E_ARG;
    return aa_map_bytes(width, height, fmt);
}


int vsr_setup_tris(const float* xyz, int64_t ntri, void* setup, int64_t setup_bytes, void* stream) {
    if (ntri < 0 || ntri > (int64_t(1) << 31)) return fail(VSR_E_ARG, "ntri %lld out of range", (long long)ntri);
    if ((ntri > 0 && !xyz) || !setup || !aligned(setup)) return fail(VSR_E_ARG, "NULL or misaligned buffer");
    if ((reinterpret_cast<uintptr_t>(xyz) & 3u) != 0) return fail(VSR_E_ARG, "vertex array not 4-byte aligned");
    int64_t need = setup_layout(ntri).bytes;
    if (setup_bytes < need)
        return fail(VSR_E_SPACE, "setup buffer %lld < %lld bytes", (long long)setup_bytes, (long long)need);
    return hip_status(launch_setup(xyz, ntri, setup, hipStream_t(stream)), "vsr_setup_tris");
}

static int check_view_buffers(const vsr_view* v, int32_t fmt) {
    if (!v) return fail(VSR_E_ARG, "view is NULL");
    if (v->width < 1 || v->height < 1 || v->width > kMaxDim || v->height > kMaxDim)
        return fail(VSR_E_ARG, "view size %dx%d outside 1..%d", v->width, v->height, kMaxDim);
    if (fmt != VSR_MAP_F32 && fmt != VSR_MAP_OCT16) return fail(VSR_E_ARG, "unknown map format %d", fmt);
    for (int q = 0; q < 9; ++q)
        if (!isfinite(v->rot[q])) return fail(VSR_E_ARG, "non-finite rotation");
    return VSR_OK;
}

int vsr_map_unpack(const vsr_view* v, int32_t fmt, const void* map, float* out, void* stream) {
    int rc = check_view_buffers(v, fmt);
    if (rc != VSR_OK) return rc;
    if (!map || !aligned(map) || !out || (reinterpret_cast<uintptr_t>(out) & 3u))
        return fail(VSR_E_ARG, "NULL or misaligned buffer");
    return hip_status(launch_map_unpack(map, v->width, v->height, fmt, rot_of(v->rot), out, hipStream_t(stream)),
                      "vsr_map_unpack");
}

int vsr_bin(const vsr_view* v, int32_t fmt, const void* map, const void* setup, int64_t ntri, int32_t bin_depth,
            uint32_t flags, void* bins, int64_t bin_bytes, void* stream) {
    int rc = check_view_buffers(v, fmt);
    if (rc != VSR_OK) return rc;
    if (!map || !setup || !bins || !aligned(map) || !aligned(setup) || !aligned(bins))
        return fail(VSR_E_ARG, "NULL or misaligned buffer");
    if (ntri < 0 || ntri > (int64_t(1) << 31)) return fail(VSR_E_ARG, "ntri out of range");
    if (bin_depth < 1 || bin_depth > kMaxDepth) return fail(VSR_E_ARG, "bin_depth %d outside 1..%d", bin_depth, kMaxDepth);
    int64_t need = bin_layout(v->width, v->height, bin_depth).bytes;
    if (bin_bytes < need) return fail(VSR_E_SPACE, "bin buffer %lld < %lld bytes", (long long)bin_bytes, (long long)need);
    if ((flags & VSR_BIN_BLOCKS) && (flags & VSR_BIN_SUPERTILES))
        return fail(VSR_E_ARG, "VSR_BIN_BLOCKS and VSR_BIN_SUPERTILES together");
    return hip_status(launch_bin(map, v->width, v->height, fmt, rot_of(v->rot), setup, ntri, bin_depth, flags, bins,
                                 hipStream_t(stream)),
                      "vsr_bin");
}

int vsr_raster(const vsr_view* v, int32_t fmt, const void* map, const void* setup, int64_t ntri, const void* bins,
               int32_t bin_depth, uint32_t* tri_id, float* depth, void* stream) {
    int rc = check_view_buffers(v, fmt);
    if (rc != VSR_OK) return rc;
    if (!map || !setup || !bins || !tri_id || !depth || !aligned(map) || !aligned(setup) || !aligned(bins))
        return fail(VSR_E_ARG, "NULL or misaligned buffer");
    if ((reinterpret_cast<uintptr_t>(tri_id) & 3u) || (reinterpret_cast<uintptr_t>(depth) & 3u))
        return fail(VSR_E_ARG, "output not 4-byte aligned");
    if (ntri < 0 || ntri > (int64_t(1) << 31)) return fail(VSR_E_ARG, "ntri out of range");
    if (bin_depth < 1 || bin_depth > kMaxDepth) return fail(VSR_E_ARG, "bin_depth %d outside 1..%d", bin_depth, kMaxDepth);
    return hip_status(launch_raster(map, v->width, v->height, fmt, rot_of(v->rot), setup, ntri, bins, bin_depth,
                                    tri_id, depth, hipStream_t(stream)),
                      "vsr_raster");
}

int vsr_raster_stats(const vsr_view* v, int32_t fmt, const void* map, const void* setup, int64_t ntri,
                     const void* bins, int32_t bin_depth, uint32_t* tri_id, float* depth, uint64_t* stats,
                     int32_t no_early_exit, void* stream) {
    int rc = check_view_buffers(v, fmt);
    if (rc != VSR_OK) return rc;
    if (!map || !setup || !bins || !tri_id || !depth || !stats || !aligned(map) || !aligned(setup) || !aligned(bins))
        return fail(VSR_E_ARG, "NULL or misaligned buffer");
    if ((reinterpret_cast<uintptr_t>(stats) & 7u) != 0) return fail(VSR_E_ARG, "stats not 8-byte aligned");
    if (ntri < 0 || ntri > (int64_t(1) << 31)) return fail(VSR_E_ARG, "ntri out of range");
    if (bin_depth < 1 || bin_depth > kMaxDepth) return fail(VSR_E_ARG, "bin_depth %d outside 1..%d", bin_depth, kMaxDepth);
    return hip_status(launch_raster(map, v->width, v->height, fmt, rot_of(v->rot), setup, ntri, bins, bin_depth,
                                    tri_id, depth, hipStream_t(stream), reinterpret_cast<unsigned long long*>(stats),
                                    no_early_exit),
                      "vsr_raster_stats");
}

static int aa_raster_common(const vsr_view* v, int32_t fmt, const void* map, const void* setup, int64_t ntri,
                            const void* bins, int32_t bin_depth, float* coverage, float* depth_pass,
                            uint32_t* dominant, uint32_t* lost, uint64_t* stats, int32_t no_skip, void* stream,
                            const char* what) {
    int rc = check_view_buffers(v, fmt);
    if (rc != VSR_OK) return rc;
    if (!map || !setup || !bins || !coverage || !depth_pass || !dominant || !aligned(map) || !aligned(setup) ||
        !aligned(bins))
        return fail(VSR_E_ARG, "NULL or misaligned buffer");
    const uintptr_t mis = reinterpret_cast<uintptr_t>(coverage) | reinterpret_cast<uintptr_t>(depth_pass) |
                          reinterpret_cast<uintptr_t>(dominant) | reinterpret_cast<uintptr_t>(lost);
    if (mis & 3u) return fail(VSR_E_ARG, "output not 4-byte aligned");
    if ((reinterpret_cast<uintptr_t>(stats) & 7u) != 0) return fail(VSR_E_ARG, "stats not 8-byte aligned");
    if (ntri < 0 || ntri > (int64_t(1) << 31)) return fail(VSR_E_ARG, "ntri out of range");
    if (bin_depth < 1 || bin_depth > kMaxDepth) return fail(VSR_E_ARG, "bin_depth %d outside 1..%d", bin_depth, kMaxDepth);
    return hip_status(launch_aa_raster(map, v->width, v->height, fmt, rot_of(v->rot), setup, ntri, bins, bin_depth,
                                       coverage, depth_pass, dominant, lost,
                                       reinterpret_cast<unsigned long long*>(stats), no_skip, hipStream_t(stream)),
                      what);
}

int vsr_aa_raster(const vsr_view* v, int32_t fmt, const void* map, const void* setup, int64_t ntri, const void* bins,
                  int32_t bin_depth, float* coverage, float* depth_pass, uint32_t* dominant, uint32_t* lost,
                  void* stream) {
    return aa_raster_common(v, fmt, map, setup, ntri, bins, bin_depth, coverage, depth_pass, dominant, lost, nullptr,
                            0, stream, "vsr_aa_raster");
}

int vsr_aa_raster_stats(const vsr_view* v, int32_t fmt, const void* map, const void* setup, int64_t ntri,
                        const void* bins, int32_t bin_depth, float* coverage, float* depth_pass, uint32_t* dominant,
                        uint32_t* lost, uint64_t* stats, int32_t no_skip, void* stream) {
    if (!stats) return fail(VSR_E_ARG, "stats is NULL");
    return aa_raster_common(v, fmt, map, setup, ntri, bins, bin_depth, coverage, depth_pass, dominant, lost, stats,
                            no_skip, stream, "vsr_aa_raster_stats");
}

int vsr_setup_particles(const float* pr, int64_t n, void* setup, int64_t setup_bytes, void* stream) {
    if (n < 0 || n > (int64_t(1) << 31)) return fail(VSR_E_ARG, "n %lld out of range", (long long)n);
    if ((n > 0 && !pr) || !setup || !aligned(setup)) return fail(VSR_E_ARG, "NULL or misaligned buffer");
    if ((reinterpret_cast<uintptr_t>(pr) & 3u) != 0) return fail(VSR_E_ARG, "particle array not 4-byte aligned");
    int64_t need = setup_layout(n).bytes;
    if (setup_bytes < need)
        return fail(VSR_E_SPACE, "setup buffer %lld < %lld bytes", (long long)setup_bytes, (long long)need);
    return hip_status(launch_setup_particles(pr, n, setup, hipStream_t(stream)), "vsr_setup_particles");
}

static int aa_particles_common(const vsr_view* v, int32_t fmt, const void* map, const void* setup, int64_t n,
                               const void* bins, int32_t bin_depth, float* coverage, float* depth_pass, float* uv,
                               uint32_t* dominant, uint32_t* lost, uint64_t* stats, int32_t no_skip, void* stream,
                               const char* what) {
    int rc = check_view_buffers(v, fmt);
    if (rc != VSR_OK) return rc;
    if (!map || !setup || !bins || !coverage || !depth_pass || !dominant || !aligned(map) || !aligned(setup) ||
        !aligned(bins))
        return fail(VSR_E_ARG, "NULL or misaligned buffer");
    const uintptr_t mis = reinterpret_cast<uintptr_t>(coverage) | reinterpret_cast<uintptr_t>(depth_pass) |
                          reinterpret_cast<uintptr_t>(dominant) | reinterpret_cast<uintptr_t>(lost) |
                          reinterpret_cast<uintptr_t>(uv);
    if (mis & 3u) return fail(VSR_E_ARG, "output not 4-byte aligned");
    if ((reinterpret_cast<uintptr_t>(stats) & 7u) != 0) return fail(VSR_E_ARG, "stats not 8-byte aligned");
    if (n < 0 || n > (int64_t(1) << 31)) return fail(VSR_E_ARG, "n out of range");
    if (bin_depth < 1 || bin_depth > kMaxDepth) return fail(VSR_E_ARG, "bin_depth %d outside 1..%d", bin_depth, kMaxDepth);
    return hip_status(launch_aa_raster(map, v->width, v->height, fmt, rot_of(v->rot), setup, n, bins, bin_depth,
                                       coverage, depth_pass, dominant, lost,
                                       reinterpret_cast<unsigned long long*>(stats), no_skip, hipStream_t(stream),
                                       kPrimParticles, uv),
                      what);
}

int vsr_aa_particles(const vsr_view* v, int32_t fmt, const void* map, const void* setup, int64_t n, const void* bins,
                     int32_t bin_depth, float* coverage, float* depth_pass, float* uv, uint32_t* dominant,
                     uint32_t* lost, void* stream) {
    return aa_particles_common(v, fmt, map, setup, n, bins, bin_depth, coverage, depth_pass, uv, dominant, lost,
                               nullptr, 0, stream, "vsr_aa_particles");
}

int vsr_aa_particles_stats(const vsr_view* v, int32_t fmt, const void* map, const void* setup, int64_t n,
                           const void* bins, int32_t bin_depth, float* coverage, float* depth_pass, float* uv,
                           uint32_t* dominant, uint32_t* lost, uint64_t* stats, int32_t no_skip, void* stream) {
    if (!stats) return fail(VSR_E_ARG, "stats is NULL");
    return aa_particles_common(v, fmt, map, setup, n, bins, bin_depth, coverage, depth_pass, uv, dominant, lost,
                               stats, no_skip, stream, "vsr_aa_particles_stats");
}

int64_t vsr_wire_bytes(int64_t ntri) {
    if (ntri < 0 || ntri > (int64_t(1) << 31)) return VSR_E_ARG;
    return wire_total_bytes(ntri);
}

int vsr_setup_wire(const void* setup, const float* xyz, int64_t ntri, void* wire, int64_t wire_bytes, void* stream) {
    if (ntri < 0 || ntri > (int64_t(1) << 31)) return fail(VSR_E_ARG, "ntri %lld out of range", (long long)ntri);
    if (!setup || !aligned(setup) || !wire || !aligned(wire) || (ntri > 0 && !xyz))
        return fail(VSR_E_ARG, "NULL or misaligned buffer");
    if ((reinterpret_cast<uintptr_t>(xyz) & 3u) != 0) return fail(VSR_E_ARG, "vertex array not 4-byte aligned");
    if (wire_bytes < vsr_wire_bytes(ntri))
        return fail(VSR_E_SPACE, "wire buffer %lld < %lld bytes", (long long)wire_bytes, (long long)vsr_wire_bytes(ntri));
    return hip_status(launch_setup_wire(setup, xyz, ntri, wire, hipStream_t(stream)), "vsr_setup_wire");
}

static int wireframe_common(const vsr_view* v, int32_t fmt, const void* map, const void* setup, const void* wire,
                            int64_t ntri, const void* bins, int32_t bin_depth, float* coverage, uint32_t* dominant,
                            uint64_t* stats, void* stream, const char* what) {
    int rc = check_view_buffers(v, fmt);
    if (rc != VSR_OK) return rc;
    if (!map || !setup || !bins || !coverage || !dominant || !wire || !aligned(map) || !aligned(setup) ||
        !aligned(bins) || !aligned(wire))
        return fail(VSR_E_ARG, "NULL or misaligned buffer");
    const uintptr_t mis = reinterpret_cast<uintptr_t>(coverage) | reinterpret_cast<uintptr_t>(dominant);
    if (mis & 3u) return fail(VSR_E_ARG, "array not 4-byte aligned");
    if ((reinterpret_cast<uintptr_t>(stats) & 7u) != 0) return fail(VSR_E_ARG, "stats not 8-byte aligned");
    if (ntri < 0 || ntri > (int64_t(1) << 31)) return fail(VSR_E_ARG, "ntri out of range");
    if (bin_depth < 1 || bin_depth > kMaxDepth) return fail(VSR_E_ARG, "bin_depth %d outside 1..%d", bin_depth, kMaxDepth);
    return hip_status(launch_wire(map, v->width, v->height, fmt, rot_of(v->rot), setup, wire, ntri, bins, bin_depth,
                                  coverage, dominant, reinterpret_cast<unsigned long long*>(stats),
                                  hipStream_t(stream)),
                      what);
}

int vsr_aa_wireframe(const vsr_view* v, int32_t fmt, const void* map, const void* setup, const void* wire,
                     int64_t ntri, const void* bins, int32_t bin_depth, float* coverage, uint32_t* dominant,
                     void* stream) {
    return wireframe_common(v, fmt, map, setup, wire, ntri, bins, bin_depth, coverage, dominant, nullptr, stream,
                            "vsr_aa_wireframe");
}

int vsr_aa_wireframe_stats(const vsr_view* v, int32_t fmt, const void* map, const void* setup, const void* wire,
                           int64_t ntri, const void* bins, int32_t bin_depth, float* coverage, uint32_t* dominant,
                           uint64_t* stats, void* stream) {
    if (!stats) return fail(VSR_E_ARG, "stats is NULL");
    return wireframe_common(v, fmt, map, setup, wire, ntri, bins, bin_depth, coverage, dominant, stats, stream,
                            "vsr_aa_wireframe_stats");
}

int64_t vsr_render_bytes(int32_t width, int32_t height) {
    if (width < 1 || height < 1 || width > kMaxDim || height > kMaxDim) return VSR_E_ARG;
    return fused_scratch_bytes(width, height);
}

int vsr_render(const vsr_view* v, int32_t fmt, const void* map, const void* setup, int64_t ntri, void* scratch,
               int64_t scratch_bytes, uint32_t* tri_id, float* depth, void* stream) {
    int rc = check_view_buffers(v, fmt);
    if (rc != VSR_OK) return rc;
    if (!map || !setup || !scratch || !tri_id || !depth || !aligned(map) || !aligned(setup) || !aligned(scratch))
        return fail(VSR_E_ARG, "NULL or misaligned buffer");
    if ((reinterpret_cast<uintptr_t>(tri_id) & 3u) || (reinterpret_cast<uintptr_t>(depth) & 3u))
        return fail(VSR_E_ARG, "output not 4-byte aligned");
    if (ntri < 0 || ntri > (int64_t(1) << 31)) return fail(VSR_E_ARG, "ntri out of range");
    int64_t need = fused_scratch_bytes(v->width, v->height);
    if (scratch_bytes < need)
        return fail(VSR_E_SPACE, "scratch %lld < %lld bytes", (long long)scratch_bytes, (long long)need);
    return hip_status(launch_fused(map, v->width, v->height, fmt, rot_of(v->rot), setup, ntri, scratch, tri_id,
                                   depth, hipStream_t(stream)),
                      "vsr_render");
}

int vsr_resolve(const vsr_view* v, int32_t fmt, const void* map, const float* xyz, int64_t ntri,
                const uint32_t* tri_id, const float* vattr, int32_t nattr, uint32_t flags, float* bary, float* attr,
                void* stream) {
    int rc = check_view_buffers(v, fmt);
    if (rc != VSR_OK) return rc;
    if (!map || !aligned(map) || !tri_id || (ntri > 0 && !xyz)) return fail(VSR_E_ARG, "NULL or misaligned buffer");
    if (ntri < 0 || ntri > (int64_t(1) << 31)) return fail(VSR_E_ARG, "ntri out of range");
    if (nattr < 0 || nattr > 64) return fail(VSR_E_ARG, "nattr %d outside 0..64", nattr);
    if (nattr > 0 && ntri > 0 && !vattr) return fail(VSR_E_ARG, "vattr is NULL");
    if ((flags & VSR_RESOLVE_NORMALIZE3) && nattr < 3) return fail(VSR_E_ARG, "NORMALIZE3 needs nattr >= 3");
    if ((flags & ~VSR_RESOLVE_NORMALIZE3) != 0) return fail(VSR_E_ARG, "unknown flags 0x%x", flags);
    const uintptr_t mis = reinterpret_cast<uintptr_t>(xyz) | reinterpret_cast<uintptr_t>(tri_id) |
                          reinterpret_cast<uintptr_t>(vattr) | reinterpret_cast<uintptr_t>(bary) |
                          reinterpret_cast<uintptr_t>(attr);
    if (mis & 3u) return fail(VSR_E_ARG, "buffer not 4-byte aligned");
    if (!bary && !attr) return VSR_OK;
    return hip_status(launch_resolve(map, v->width, v->height, fmt, rot_of(v->rot), xyz, ntri, tri_id, vattr, nattr,
                                     (flags & VSR_RESOLVE_NORMALIZE3) != 0, bary, nattr > 0 ? attr : nullptr,
                                     hipStream_t(stream)),
                      "vsr_resolve");
}

int64_t vsr_resolve_pack_bytes(int64_t ntri, int32_t nattr) {
    if (ntri < 0 || ntri > (int64_t(1) << 31) || nattr < 0 || nattr > 64) return VSR_E_ARG;
    const int64_t b = ntri * int64_t(resolve_stride(nattr)) * 4;
    return align256(b > 0 ? b : 256);
}

int vsr_resolve_pack(const float* xyz, const float* vattr, int64_t ntri, int32_t nattr, void* packed,
                     int64_t packed_bytes, void* stream) {
    if (ntri < 0 || ntri > (int64_t(1) << 31)) return fail(VSR_E_ARG, "ntri out of range");
    if (nattr < 0 || nattr > 64) return fail(VSR_E_ARG, "nattr %d outside 0..64", nattr);
    if (!packed || !aligned(packed) || (ntri > 0 && (!xyz || (nattr > 0 && !vattr))))
        return fail(VSR_E_ARG, "NULL or misaligned buffer");
    if ((reinterpret_cast<uintptr_t>(xyz) | reinterpret_cast<uintptr_t>(vattr)) & 3u)
        return fail(VSR_E_ARG, "buffer not 4-byte aligned");
    const int64_t need = vsr_resolve_pack_bytes(ntri, nattr);
    if (packed_bytes < need)
        return fail(VSR_E_SPACE, "packed buffer %lld < %lld bytes", (long long)packed_bytes, (long long)need);
    return hip_status(launch_resolve_pack(xyz, vattr, ntri, nattr, packed, hipStream_t(stream)), "vsr_resolve_pack");
}

int vsr_resolve_packed(const vsr_view* v, int32_t fmt, const void* map, const void* packed, int64_t ntri,
                       int32_t nattr, const uint32_t* tri_id, uint32_t flags, float* bary, float* attr, void* stream) {
    int rc = check_view_buffers(v, fmt);
    if (rc != VSR_OK) return rc;
    if (!map || !aligned(map) || !tri_id || !packed || !aligned(packed))
        return fail(VSR_E_ARG, "NULL or misaligned buffer");
    if (ntri < 0 || ntri > (int64_t(1) << 31)) return fail(VSR_E_ARG, "ntri out of range");
    if (nattr < 0 || nattr > 64) return fail(VSR_E_ARG, "nattr %d outside 0..64", nattr);
    if ((flags & VSR_RESOLVE_NORMALIZE3) && nattr < 3) return fail(VSR_E_ARG, "NORMALIZE3 needs nattr >= 3");
    if ((flags & ~VSR_RESOLVE_NORMALIZE3) != 0) return fail(VSR_E_ARG, "unknown flags 0x%x", flags);
    const uintptr_t mis = reinterpret_cast<uintptr_t>(tri_id) | reinterpret_cast<uintptr_t>(bary) |
                          reinterpret_cast<uintptr_t>(attr);
    if (mis & 3u) return fail(VSR_E_ARG, "buffer not 4-byte aligned");
    if (!bary && !attr) return VSR_OK;
    return hip_status(launch_resolve(map, v->width, v->height, fmt, rot_of(v->rot), nullptr, ntri, tri_id, nullptr,
                                     nattr, (flags & VSR_RESOLVE_NORMALIZE3) != 0, bary, nattr > 0 ? attr : nullptr,
                                     hipStream_t(stream), packed),
                      "vsr_resolve_packed");
}

int64_t vsr_submit_bytes(const vsr_job* jobs, int32_t njobs, int32_t fmt, int32_t mode, int32_t bin_depth) {
    if (!jobs || njobs < 1 || njobs > 4096) return VSR_E_ARG;
    if (fmt != VSR_MAP_F32 && fmt != VSR_MAP_OCT16) return VSR_E_ARG;
    mode &= ~(VSR_SUBMIT_TABLE_READY | VSR_SUBMIT_BIN_BLOCKS | VSR_SUBMIT_BIN_SUPERTILES | VSR_SUBMIT_BIN_TILE16 |
              VSR_SUBMIT_PERSISTENT);
    if (mode != VSR_SUBMIT_BINNED && mode != VSR_SUBMIT_FUSED) return VSR_E_ARG;
    if (mode == VSR_SUBMIT_BINNED && (bin_depth < 1 || bin_depth > kMaxDepth)) return VSR_E_ARG;
    for (int32_t q = 0; q < njobs; ++q) {
        const vsr_view& v = jobs[q].view;
        if (v.width < 1 || v.height < 1 || v.width > kMaxDim || v.height > kMaxDim) return VSR_E_ARG;
    }
    return submit_bytes(jobs, njobs, fmt, mode, bin_depth);
}

int64_t vsr_submit_table_bytes(int32_t njobs) {
    if (njobs < 1 || njobs > 4096) return VSR_E_ARG;
    return submit_table_bytes(njobs);
}

int64_t vsr_submit_table_offset(void) { return submit_table_offset(); }

int vsr_submit_table(const vsr_job* jobs, int32_t njobs, int32_t fmt, int32_t mode, int32_t bin_depth,
                     const void* workspace, void* host_table, int64_t host_table_bytes) {
    if (!jobs || njobs < 1 || njobs > 4096) return fail(VSR_E_ARG, "njobs %d outside 1..4096", njobs);
    if (!workspace || !aligned(workspace) || !host_table) return fail(VSR_E_ARG, "NULL or misaligned buffer");
    if (host_table_bytes < submit_table_bytes(njobs)) return fail(VSR_E_SPACE, "host table too small");
    mode &= ~(VSR_SUBMIT_TABLE_READY | VSR_SUBMIT_BIN_BLOCKS | VSR_SUBMIT_BIN_SUPERTILES | VSR_SUBMIT_BIN_TILE16 |
              VSR_SUBMIT_PERSISTENT);
    for (int32_t q = 0; q < njobs; ++q) {
        MapParams P;
        int rc = make_map_params(&jobs[q].view, fmt, 0, &P, nullptr);
        if (rc != VSR_OK) return rc;
    }
    submit_table(jobs, njobs, fmt, mode, bin_depth, const_cast<void*>(workspace), host_table);
    return VSR_OK;
}

static int submit_common(const vsr_job* jobs, int32_t njobs, int32_t fmt, int32_t mode, int32_t bin_depth,
                         void* workspace, int64_t ws_bytes, hipEvent_t* ev, void* stream, const char* what) {
    const bool table_ready = (mode & VSR_SUBMIT_TABLE_READY) != 0;
    uint32_t shape = 0;
    if (mode & VSR_SUBMIT_BIN_BLOCKS) shape |= VSR_BIN_BLOCKS;
    if (mode & VSR_SUBMIT_BIN_SUPERTILES) shape |= VSR_BIN_SUPERTILES;
    if (mode & VSR_SUBMIT_BIN_TILE16) shape |= VSR_BIN_TILE16;
    if (mode & VSR_SUBMIT_PERSISTENT) shape |= kShapePersistent;
    if ((shape & ~kShapePersistent) == (VSR_BIN_BLOCKS | VSR_BIN_SUPERTILES))
        return fail(VSR_E_ARG, "VSR_SUBMIT_BIN_BLOCKS and VSR_SUBMIT_BIN_SUPERTILES together");
    mode &= ~(VSR_SUBMIT_TABLE_READY | VSR_SUBMIT_BIN_BLOCKS | VSR_SUBMIT_BIN_SUPERTILES | VSR_SUBMIT_BIN_TILE16 |
              VSR_SUBMIT_PERSISTENT);
    if (!jobs || njobs < 1 || njobs > 4096) return fail(VSR_E_ARG, "njobs %d outside 1..4096", njobs);
    if (mode != VSR_SUBMIT_BINNED && mode != VSR_SUBMIT_FUSED) return fail(VSR_E_ARG, "unknown submit mode %d", mode);
    if (mode == VSR_SUBMIT_BINNED && (bin_depth < 1 || bin_depth > kMaxDepth))
        return fail(VSR_E_ARG, "bin_depth %d outside 1..%d", bin_depth, kMaxDepth);
    if (!workspace || !aligned(workspace)) return fail(VSR_E_ARG, "workspace NULL or misaligned");
    for (int32_t q = 0; q < njobs; ++q) {
        const vsr_job& J = jobs[q];
        MapParams P;
        int rc = make_map_params(&J.view, fmt, 0, &P, nullptr);
        if (rc != VSR_OK) return rc;
        if (!J.setup || !aligned(J.setup) || !J.tri_id || !J.depth || J.ntri < 0 || J.ntri > (int64_t(1) << 31))
            return fail(VSR_E_ARG, "job %d: bad scene or output pointer", q);
        if ((reinterpret_cast<uintptr_t>(J.tri_id) & 3u) || (reinterpret_cast<uintptr_t>(J.depth) & 3u))
            return fail(VSR_E_ARG, "job %d: output not 4-byte aligned", q);
    }
    int64_t need = submit_bytes(jobs, njobs, fmt, mode, bin_depth);
    if (ws_bytes < need) return fail(VSR_E_SPACE, "workspace %lld < %lld bytes", (long long)ws_bytes, (long long)need);
    return hip_status(
        launch_submit(jobs, njobs, fmt, mode, bin_depth, workspace, table_ready, shape, hipStream_t(stream), ev),
                      what);
}

int vsr_submit(const vsr_job* jobs, int32_t njobs, int32_t fmt, int32_t mode, int32_t bin_depth, void* workspace,
               int64_t ws_bytes, void* stream) {
    return submit_common(jobs, njobs, fmt, mode, bin_depth, workspace, ws_bytes, nullptr, stream, "vsr_submit");
}

int vsr_submit_timed(const vsr_job* jobs, int32_t njobs, int32_t fmt, int32_t mode, int32_t bin_depth,
                     void* workspace, int64_t ws_bytes, void* const* events, int32_t nevents, void* stream) {
    if (!events || nevents != 4) return fail(VSR_E_ARG, "vsr_submit_timed needs 4 events, got %d", nevents);
    hipEvent_t ev[4];
    for (int q = 0; q < 4; ++q) {
        if (!events[q]) return fail(VSR_E_ARG, "event %d is NULL", q);
        ev[q] = reinterpret_cast<hipEvent_t>(events[q]);
    }
    return submit_common(jobs, njobs, fmt, mode, bin_depth, workspace, ws_bytes, ev, stream, "vsr_submit_timed");
}

int vsr_calib_copy(const void* src, void* dst, int64_t nbytes, void* stream) {
    if (!src || !dst || !aligned(src) || !aligned(dst)) return fail(VSR_E_ARG, "NULL or misaligned buffer");
    if (nbytes < 16 || (nbytes & 15)) return fail(VSR_E_ARG, "nbytes %lld not a positive multiple of 16", (long long)nbytes);
    return hip_status(launch_calib_copy(src, dst, nbytes, hipStream_t(stream)), "vsr_calib_copy");
}

int vsr_calib_fma(float* out, int64_t nthreads, int32_t iters, void* stream) {
    if (!out || (reinterpret_cast<uintptr_t>(out) & 3u)) return fail(VSR_E_ARG, "NULL or misaligned buffer");
    if (nthreads < 256 || (nthreads & 255) || nthreads / 256 > 0x7FFFFFFF)
        return fail(VSR_E_ARG, "nthreads %lld not a positive multiple of 256", (long long)nthreads);
    if (iters < 1) return fail(VSR_E_ARG, "iters %d < 1", iters);
    return hip_status(launch_calib_fma(out, nthreads, iters, hipStream_t(stream)), "vsr_calib_fma");
}

int vsr_bin_overflow(const void* bins_or_ws, int32_t is_workspace, int64_t* overflowed_tiles) {
    (void)is_workspace;  // both keep the overflow counter in their first word
    if (!bins_or_ws || !overflowed_tiles) return fail(VSR_E_ARG, "NULL argument");
    uint32_t w = 0;
    hipError_t e = hipMemcpy(&w, bins_or_ws, 4, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_status(e, "vsr_bin_overflow");
    *overflowed_tiles = w;
    return VSR_OK;
}

const char* vsr_strerror(int code) {
    switch (code) {
    case VSR_OK: return "ok";
    case VSR_E_ARG: return "invalid argument";
    case VSR_E_SPACE: return "buffer too small";
    case VSR_E_RANGE: return "view parameters outside the limits";
    case VSR_E_HIP: return "HIP runtime error";
    default: return "unknown error";
    }
}

const char* vsr_last_error(void) { return g_err; }

}  // extern "C"
