/*
 * vsr — visual-sphere perspective-map rasterization on AMD Instinct MI355X
 * (gfx950).  C ABI of libvsr.so.
 *
 * The method (J. M. Fober, "Perspective picture from Visual Sphere: a new
 * approach to image rasterization"): every pixel of a picture owns a unit
 * view direction G taken from a perspective vector map (section 2.1.2,
 * Universal Perspective model with parameters k, l, s and angle of view
 * Omega).  A triangle ABC seen from the projection origin O covers the
 * pixel when G lies on the inner side of the three great-circle planes
 * through O that contain its edges, i.e. when G.(AxB), G.(BxC), G.(CxA) all
 * pass the binary step (sections 1.1 and 1.1.1).  The covered fragment's
 * depth is the ray-plane distance r = A.N / G.N with N the triangle's hard
 * normal (section 1.1.4), and the nearest depth wins (depth-pass test,
 * section 1.4).
 *
 * Conventions shared by every call
 *   - All buffer pointers are DEVICE pointers owned by the caller.  The
 *     library never allocates or frees device memory and keeps no device
 *     state between calls (the one exception is the scratch array of
 *     vsr_render_noalloc, part of the loaded code object).  Buffer sizes
 *     come from the vsr_*_bytes() functions; buffers must be 256-byte
 *     aligned.
 *   - `stream` is a hipStream_t passed as void* (NULL = default stream).
 *     Every call only enqueues work on it and returns; results are ready
 *     when the stream is synchronised.
 *   - Return value: VSR_OK (0) or a negative VSR_E_* code; on error nothing
 *     has been enqueued and vsr_last_error() describes the cause (the text
 *     is per thread).  No C++ exception crosses this ABI.
 *   - Output images are row-major, top row first: pixel (i, j) (column i,
 *     row j) is element j*width + i.
 *   - Triangle ids are column indices of the input vertex array.
 *   - Calls on distinct streams with distinct buffers may run concurrently.
 */
#ifndef VSR_H
#define VSR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- codes */
#define VSR_OK 0
#define VSR_E_ARG (-1)   /* null pointer, bad size or dimension, misaligned   */
#define VSR_E_SPACE (-2) /* a buffer is smaller than its vsr_*_bytes() size    */
#define VSR_E_RANGE (-3) /* view parameters outside the limits (VSR_STRICT)    */
#define VSR_E_HIP (-4)   /* the HIP runtime refused a launch                   */

/* map storage formats */
#define VSR_MAP_F32 0   /* three float planes (x, y, z): 12 bytes per pixel   */
#define VSR_MAP_OCT16 1 /* octahedral unit vector, two fp16: 4 bytes per pixel */

/* vsr_build_map flags */
#define VSR_STRICT 1u /* reject parameters outside the limits instead of clamping */
#define VSR_MAP_AA 2u       /* also store the global delta and widen the caps: see vsr_aa_raster   */
#define VSR_MAP_AA_LINES 4u /* VSR_MAP_AA with caps widened for wire frames: see vsr_aa_wireframe */

/* angle-of-view types (section 2, remark on normalising 2D coordinates) */
#define VSR_AOV_HORIZONTAL 0
#define VSR_AOV_DIAGONAL 1
#define VSR_AOV_VERTICAL 2
#define VSR_AOV_HORIZONTAL_4X3 3

/* vsr_bin flags */
#define VSR_BIN_ALL 1u /* list every live triangle in every tile (no culling) */
/* Workgroup shape of the binner (the lists are the same either way):
 * candidates gathered once per 32x32-pixel block of 4x4 tiles, or once per
 * 16x16 super-tile of 2x2 tiles.  Blocks need a list capacity (bin_depth
 * rounded up to a power of two, at least 64) of at most 256: above it
 * super-tiles are used whatever the flags.  Neither flag: blocks when the
 * launch has at least 2560 of them, super-tiles otherwise. */
#define VSR_BIN_BLOCKS 2u
#define VSR_BIN_SUPERTILES 4u
/* Bin tile edge 16 instead of 8: one list per 16x16 super-tile (2x2 tiles),
 * of the triangles that may meet the super-tile, written once in
 * depth-bucket order (fewer, longer lists: about half the entries at
 * 1080p x 1M).  vsr_raster reads the tile edge from the bin buffer and
 * keeps, for each 8x8 tile, the entries that pass the 8x8 binner's own tile
 * test, so images are identical either way.  A list longer than bin_depth
 * overflows as a whole super-tile.  With 16x16 lists the 32x32-block shape
 * takes list capacities up to 1024. */
#define VSR_BIN_TILE16 8u

#define VSR_NO_HIT 0xFFFFFFFFu /* tri_id of a pixel that nothing covers */

/* Edge of the square pixel tiles that maps and the rasterizer use (bins:
 * VSR_TILE, or 16 with VSR_BIN_TILE16). */
#define VSR_TILE 8

/* One view request (host memory).
 *   width, height  picture size in pixels, 1..32768 each.
 *   aov            VSR_AOV_* angle-of-view type.
 *   k, l, s        Universal Perspective projection type, cylindricity and
 *                  anamorphic correction (section 2.1.1).
 *   omega_deg      angle of view in degrees.
 *   rot            camera->world rotation, row-major 3x3; the camera looks
 *                  along +z with +x right and +y down the picture. */
typedef struct {
    int32_t width, height, aov, reserved;
    float k, l, s, omega_deg;
    float rot[9];
} vsr_view;

/* ------------------------------------------------------------- sizing */

/* Bytes of a perspective map of a width x height view in format fmt
 * (VSR_MAP_*), including its per-tile bounding caps.  <0 on bad input. */
int64_t vsr_map_bytes(int32_t width, int32_t height, int32_t fmt);

/* Bytes of the setup buffer for ntri triangles (records, bounding caps,
 * direction index and the scratch space the setup sorts use).  <0 on bad
 * input. */
int64_t vsr_setup_bytes(int64_t ntri);

/* Bytes of the bin buffer of a width x height view with lists of at most
 * bin_depth triangles per tile (1..2048).  <0 on bad input. */
int64_t vsr_bin_bytes(int32_t width, int32_t height, int32_t bin_depth);

/* ------------------------------------------------------------ pipeline */

/* Step 1 — perspective vector map (sections 2, 2.1.1, 2.1.2).
 * Applies the parameter limits of section 2.1.1 (or, with VSR_STRICT,
 * returns VSR_E_RANGE when a parameter is outside them), computes the unit
 * world direction of every pixel centre ((i+1/2)/W, (j+1/2)/H), and the
 * bounding cap of every tile.  Pixels outside the projection's domain
 * (k < 0 with |sin(k*Omega/2)*R| > 1) get no direction and are never
 * covered.
 *   v           view (host).
 *   fmt         VSR_MAP_F32 or VSR_MAP_OCT16.
 *   map         device buffer of vsr_map_bytes(width, height, fmt) bytes.
 *   v_effective optional host output: the view after clamping. */
int vsr_build_map(const vsr_view* v, int32_t fmt, uint32_t flags, void* map, int64_t map_bytes,
                  vsr_view* v_effective, void* stream);

/* Other map generators (sections 2.2.2-2.2.4, 2.2.7-2.2.9) and lens
 * distortion (section 2.3).  A vsr_lens picks the generator; the view's
 * width, height and rotation always apply, its k, l, s, omega_deg and aov
 * only to VSR_LENS_UNIVERSAL.  Parameters (p[]):
 *   VSR_LENS_UNIVERSAL  p[0..5] = k1, k2, p1, p2, q1, q2: Brown-Conrady
 *                       distortion (radial, thin prism, decentering) of the
 *                       view coordinates before the 2D->3D transform; all
 *                       zero = vsr_build_map.
 *   VSR_LENS_EQUIRECT   none: longitude pi (2fs - 1) across, polar angle
 *                       pi ft from straight up down the picture.
 *   VSR_LENS_CUBE       none: six 90-degree faces side by side (face
 *                       floor(6 fs): +x, -x, -z, +z, +y, -y).
 *   VSR_LENS_SCREENS    n = screens (1..64), p[0] = one screen's horizontal
 *                       angle of view in degrees (0, 180); screen s is
 *                       turned about the vertical axis by (s - (n-1)/2) p[0].
 *   VSR_LENS_VR         p[0] = vertical angle of view (0, 180) degrees,
 *                       p[1] = interpupillary distance in screen widths,
 *                       p[2], p[3] = radial lens coefficients k1, k2 (the
 *                       factor (1 + k1 R^2 + k2 R^4)/(1 + k1 + k2);
 *                       1 + k1 + k2 = 0 is refused); left eye on the left.
 *   VSR_LENS_PANORAMA   p[0] = horizontal angle of view (0, 360] degrees of
 *                       a unit cylinder; its height follows from W/H.
 *   VSR_LENS_DOME       p[0] = compression angle [-89, 90] degrees, p[1] =
 *                       tilt in degrees, p[2] = view position offset in
 *                       dome radii (-1, 1): full-dome fisheye (section
 *                       2.2.3), zenith +y at the picture centre, 90 degrees
 *                       + compression at the inscribed circle; pixels
 *                       outside that circle have no direction.
 * The map has the same layout as vsr_build_map's (flags: VSR_STRICT for the
 * Universal parameters, VSR_MAP_AA), and every later step takes it
 * unchanged.  VSR_E_ARG for an unknown type or parameters outside the
 * ranges above. */
#define VSR_LENS_UNIVERSAL 0
#define VSR_LENS_EQUIRECT 1
#define VSR_LENS_CUBE 2
#define VSR_LENS_SCREENS 3
#define VSR_LENS_VR 4
#define VSR_LENS_PANORAMA 5
#define VSR_LENS_DOME 6
typedef struct {
    int32_t type, n;
    float p[8];
} vsr_lens;
int vsr_build_map_lens(const vsr_view* v, const vsr_lens* lens, int32_t fmt, uint32_t flags, void* map,
                       int64_t map_bytes, vsr_view* v_effective, void* stream);

/* Copy a map's directions out to a row-major device array
 * out[(j*width + i)*3 + c] (float; all zero for a pixel without a direction),
 * decoding VSR_MAP_OCT16.  For inspection and tests; not on the hot path. */
int vsr_map_unpack(const vsr_view* v, int32_t fmt, const void* map, float* out, void* stream);

/* Step 2 — per-triangle setup (sections 1.1, 1.1.2, 1.1.4).
 *   xyz     device float[9][ntri] structure of arrays: rows ax, ay, az, bx,
 *           by, bz, cx, cy, cz; vertices relative to the projection origin.
 *   setup   device buffer of vsr_setup_bytes(ntri) bytes; it receives the
 *           oriented unit edge-plane normals, the oriented unit plane normal
 *           and plane distance, a bounding cap (section 1.1.2) and a depth
 *           lower bound per triangle, sorted nearest first, plus a
 *           multi-level cube-map index of the caps.
 * Triangles whose plane passes through O (det[A,B,C] = 0 in FP32, to a
 * relative 1e-7) cover nothing.  The setup depends only on the vertices, so
 * one setup serves every view rendered from the same origin. */
int vsr_setup_tris(const float* xyz, int64_t ntri, void* setup, int64_t setup_bytes, void* stream);

/* Step 3 — conservative binning (the coarse "once per region" test of
 * section 1.1.3, made conservative).  For every tile of the map it lists
 * the triangles whose bounding cap meets the tile's cap and whose three edge
 * planes do not exclude the whole tile, nearest first.  A tile with more
 * than bin_depth candidates is marked overflowed; vsr_raster then gathers
 * its candidates itself, so overflow costs time, never pixels.
 *   v, fmt, map  the map built by vsr_build_map for this view.
 *   setup, ntri  the setup buffer of vsr_setup_tris.
 *   bins         device buffer of vsr_bin_bytes(width, height, bin_depth). */
int vsr_bin(const vsr_view* v, int32_t fmt, const void* map, const void* setup, int64_t ntri,
            int32_t bin_depth, uint32_t flags, void* bins, int64_t bin_bytes, void* stream);

/* Step 4 — rasterization with depth test (sections 1.1, 1.1.1, 1.1.4, 1.4).
 * Every pixel tests its direction against the edge planes of every listed
 * triangle (strict > 0), takes r = d / (G.N) for covered ones and keeps the
 * smallest (r, triangle id) pair.
 *   tri_id  device uint32[height][width]; VSR_NO_HIT where nothing covers.
 *   depth   device float[height][width]; +inf where nothing covers.  Depth
 *           is the distance along the unit view direction, not z. */
int vsr_raster(const vsr_view* v, int32_t fmt, const void* map, const void* setup, int64_t ntri,
               const void* bins, int32_t bin_depth, uint32_t* tri_id, float* depth, void* stream);

/* Instrumented vsr_raster (same images) that also counts, into the device
 * array stats[4] of uint64: executed pixel-triangle tests (pixels with a
 * direction x triangles processed), covered fragments processed, triangles
 * processed, tiles.  With no_early_exit != 0 every listed triangle is
 * processed, so stats[1] is then the number of covered (pixel, triangle)
 * pairs of the frame.  For measurement; slower than vsr_raster. */
int vsr_raster_stats(const vsr_view* v, int32_t fmt, const void* map, const void* setup, int64_t ntri,
                     const void* bins, int32_t bin_depth, uint32_t* tri_id, float* depth, uint64_t* stats,
                     int32_t no_early_exit, void* stream);

/* Steps 3+4 fused for one view: bytes of the scratch buffer vsr_render
 * needs for a width x height view. */
int64_t vsr_render_bytes(int32_t width, int32_t height);

/* Steps 3+4 fused, depth-sliced (same images as vsr_bin + vsr_raster, bit
 * for bit).  Triangles are visited nearest-first in slices; a 16x16 block of
 * pixels gathers a slice's candidates into on-chip lists, rasterizes them,
 * and stops as soon as every pixel is nearer than the next slice can be, so
 * occluded geometry is never gathered.
 *   scratch  device buffer of vsr_render_bytes(width, height) bytes. */
int vsr_render(const vsr_view* v, int32_t fmt, const void* map, const void* setup, int64_t ntri, void* scratch,
               int64_t scratch_bytes, uint32_t* tri_id, float* depth, void* stream);

/* vsr_render for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same kernel and images as vsr_render, with its list scratch taken from a
 * device array the library holds (VSR_NOALLOC_MAX_TILES x 4 KiB = 128 MiB
 * on every GPU that loads the library, until the process ends) instead of a
 * caller buffer.  The call allocates nothing.  Views of more than
 * VSR_NOALLOC_MAX_TILES tiles of 8x8 pixels (1920x1080 has 32,400) are
 * refused with VSR_E_SPACE.  All calls on one GPU share its array and the
 * array keeps the last call's contents: calls that overlap in time on one GPU
 * (other streams, other threads) race on it and may give wrong images;
 * serialise them.  The current device must be the device of `stream`.
 * Other arguments and errors as vsr_render. */
#define VSR_NOALLOC_MAX_TILES 32768
int vsr_render_noalloc(const vsr_view* v, int32_t fmt, const void* map, const void* setup, int64_t ntri,
                       uint32_t* tri_id, float* depth, void* stream);

/* Step 6 — fragment data from barycentric coordinates (section 1.1.4,
 * second half).  For every pixel whose tri_id names a triangle: the
 * barycentric weights (b_A, b_B, b_C) of the point where the pixel's ray
 * meets that triangle's plane (they sum to 1, all >= 0 inside), and per
 * vertex data interpolated with them, f = b_A A_f + b_B B_f + b_C C_f
 * (perspective-correct: the weights are those of the 3D point).  With
 * VSR_RESOLVE_NORMALIZE3 the first three data components are normalised
 * (the normal pass).  Pixels with no hit, no direction, or a ray parallel
 * to the plane get zeros.
 *   v, fmt, map  the view and its map (any map of the same lens).
 *   xyz, ntri    the device triangle array given to vsr_setup_tris
 *                (float[9][ntri]).
 *   tri_id       device uint32[height][width] from vsr_raster / vsr_render.
 *   vattr        device float[3][nattr][ntri]: data of vertex v (0=A, 1=B,
 *                2=C), component k, triangle t at (v*nattr + k)*ntri + t;
 *                may be NULL when nattr == 0.  nattr: 0..64.
 *   bary         device float[3][height][width] or NULL.
 *   attr         device float[nattr][height][width] or NULL.
 * Returns VSR_E_ARG for bad sizes or pointers, or NORMALIZE3 with nattr < 3. */
#define VSR_RESOLVE_NORMALIZE3 1u
int vsr_resolve(const vsr_view* v, int32_t fmt, const void* map, const float* xyz, int64_t ntri,
                const uint32_t* tri_id, const float* vattr, int32_t nattr, uint32_t flags, float* bary, float* attr,
                void* stream);

/* Step 7 — aliasing-free coverage (sections 1.1.1, 1.1.2, 1.4).
 *
 * Bytes of a map built with VSR_MAP_AA: the map of vsr_map_bytes followed by
 * one float per pixel (the global delta).  <0 on bad input. */
int64_t vsr_aa_map_bytes(int32_t width, int32_t height, int32_t fmt);

/* Anti-aliased coverage and front-to-back combination.  Per pixel and
 * triangle the fragment mask is
 *   m = min(gpstep(n_0.G), gpstep(n_1.G), gpstep(n_2.G), gpstep(miter)),
 *   gpstep(x) = clamp(delta*x + 1/2, 0, 1)      (section 1.1.1)
 * with n_i the oriented unit edge-plane normals, delta the pixel's global
 * delta (1 / largest component of fwidth of the camera-frame map, by
 * central differences), and miter = (S.G - |S|)/sin(rho) for the smallest
 * circle (S, rho) of section 1.1.2 (divided by sin rho so that its slope is
 * one pixel wide like the edges').  Fragments with m > 0 whose plane is in
 * front (r = d/(G.N) > 0) are combined nearest first by (r, id), as in
 * section 1.4: m_fc = min(m, 1 - m_b), m_b += m_fc, depth += m_fc * r.
 *   map          built by vsr_build_map with VSR_MAP_AA into a buffer of
 *                vsr_aa_map_bytes(width, height, fmt) bytes; its tile caps
 *                are widened by the pixel step's fringe, so vsr_bin on it
 *                lists every triangle whose mask is non-zero in a tile.
 *   setup, ntri  from vsr_setup_tris; bins, bin_depth from vsr_bin on map
 *                (an overflowed tile gathers its own candidates).
 *   coverage     device float[height][width]: m_b in [0, 1] (0: no hit or
 *                no direction).
 *   depth_pass   device float[height][width]: sum of m_fc * r (the depth
 *                pass, not divided by the coverage).
 *   dominant     device uint32[height][width]: the triangle with the largest
 *                clipped share m_fc (ties: the nearer), VSR_NO_HIT if none.
 *   lost         optional device uint32 (may be NULL): receives the number
 *                of pixels that met more than 8 fragments before their masks
 *                saturated; only those pixels can differ from the exact
 *                combination.
 * A map built without VSR_MAP_AA gives undefined images (no delta plane). */
int vsr_aa_raster(const vsr_view* v, int32_t fmt, const void* map, const void* setup, int64_t ntri, const void* bins,
                  int32_t bin_depth, float* coverage, float* depth_pass, uint32_t* dominant, uint32_t* lost,
                  void* stream);

/* Instrumented vsr_aa_raster (same images) that also counts, into the device
 * array stats[4] of uint64: pixel-triangle mask evaluations (pixels with a
 * direction x triangles tested), fragments (m > 0, plane in front) found,
 * triangles skipped by the wave's saturation-depth test, tiles.  With
 * no_skip != 0 every listed triangle is tested, so stats[1] is then the
 * number of (pixel, triangle) fragments of the frame at all depths.  For
 * measurement; slower than vsr_aa_raster. */
int vsr_aa_raster_stats(const vsr_view* v, int32_t fmt, const void* map, const void* setup, int64_t ntri,
                        const void* bins, int32_t bin_depth, float* coverage, float* depth_pass, uint32_t* dominant,
                        uint32_t* lost, uint64_t* stats, int32_t no_skip, void* stream);

/* Step 8 — wire frame of the triangles' sides (section 1.2), aliasing-free.
 * Per pixel and side P->Q of every listed live triangle: the line step of
 * the side's great circle with the global delta, h = 1 - min(|n.G| delta, 1)
 * (a strip one pixel wide each way), limited by the pixel step of the cap
 * around the segment (centre |P_hat + Q_hat|, cos of the radius
 * |(P_hat + Q_hat)/2|; value divided by sin of the radius).  Lines do not
 * hide each other: coverage is the largest mask over all sides and dominant
 * the triangle of that side (ties: the lower id; VSR_NO_HIT where nothing
 * draws).
 *   map          built with VSR_MAP_AA_LINES (caps widened by 5/4 pixel:
 *                a side draws up to sqrt(5)/2 pixel from its segment);
 *                bins from vsr_bin on that map and the triangles' setup.
 *   wire, ntri   the side caps of the scene from vsr_setup_wire.
 *   coverage     device float[height][width]; dominant uint32[height][width]. */
int vsr_aa_wireframe(const vsr_view* v, int32_t fmt, const void* map, const void* setup, const void* wire,
                     int64_t ntri, const void* bins, int32_t bin_depth, float* coverage, uint32_t* dominant,
                     void* stream);
/* Bytes of the side-cap buffer of ntri triangles: 64 per triangle of caps
 * (rounded up to 256), then 4 per triangle of scratch for vsr_setup_wire
 * (rounded up to 256).  <0 on bad input. */
int64_t vsr_wire_bytes(int64_t ntri);
/* Side caps of a scene for vsr_aa_wireframe, once per scene after
 * vsr_setup_tris (again whenever the setup is redone): per triangle, in the
 * setup's nearest-first order, each side's cap centre and the two
 * constants of its pixel step, and the triangle id.
 *   setup, xyz, ntri  the setup buffer and the vertex array given to it.
 *   wire              device buffer of vsr_wire_bytes(ntri) bytes. */
int vsr_setup_wire(const void* setup, const float* xyz, int64_t ntri, void* wire, int64_t wire_bytes, void* stream);
/* Instrumented vsr_aa_wireframe: stats[4] of uint64 receive (pixels with a
 * direction x triangles tested, (pixel, triangle) pairs with a mask > 0, 0,
 * tiles). */
int vsr_aa_wireframe_stats(const vsr_view* v, int32_t fmt, const void* map, const void* setup, const void* wire,
                           int64_t ntri, const void* bins, int32_t bin_depth, float* coverage, uint32_t* dominant,
                           uint64_t* stats, void* stream);

/* Step 9 — procedural particles (section 1.3), aliasing-free, combined
 * front to back (section 1.4).
 * vsr_setup_particles prepares n spheres pr = device float[4][n] (rows x, y,
 * z, radius; positions relative to O) into a setup buffer of
 * vsr_setup_bytes(n) bytes, in the same layout as triangles (vsr_bin bins
 * them unchanged; vsr_raster draws nothing for them).  A particle with
 * radius <= 0 or containing O is skipped. */
int vsr_setup_particles(const float* pr, int64_t n, void* setup, int64_t setup_bytes, void* stream);
/* Per pixel and particle: mask = pixel step of (G.P_hat - cos rho)/sin rho,
 * sin rho = r/|P| (the sphere's silhouette cone); depth where the ray meets
 * the particle's plane (through P, normal P_hat), |P| / (G.P_hat); texture
 * coordinates (G.X, G.Y) |P|/(2r) + 1/2 with X = |(P_z, 0, -P_x)| (the x
 * axis for a vertical P) and Y = X x P_hat.  Fragments are combined nearest
 * first by (depth, id) as in vsr_aa_raster; the texture coordinates as a
 * pass like the depth (section 1.4).
 *   map          built with VSR_MAP_AA; bins from vsr_bin on it and the
 *                particles' setup.
 *   uv           optional device float[2][height][width] (u plane, then v).
 *   other outputs and lost as in vsr_aa_raster. */
int vsr_aa_particles(const vsr_view* v, int32_t fmt, const void* map, const void* setup, int64_t n, const void* bins,
                     int32_t bin_depth, float* coverage, float* depth_pass, float* uv, uint32_t* dominant,
                     uint32_t* lost, void* stream);
/* Instrumented vsr_aa_particles (stats as in vsr_aa_raster_stats). */
int vsr_aa_particles_stats(const vsr_view* v, int32_t fmt, const void* map, const void* setup, int64_t n,
                           const void* bins, int32_t bin_depth, float* coverage, float* depth_pass, float* uv,
                           uint32_t* dominant, uint32_t* lost, uint64_t* stats, int32_t no_skip, void* stream);

/* Fragment data from a packed copy of the scene.  vsr_resolve gathers a
 * winner's 9 coordinates and 3*nattr data values from rows of the [9][T] and
 * [3][K][T] arrays, each in its own memory line; the packed form keeps one
 * triangle's vertices and data in one row (A, B, C, then vertex v's
 * component k at 9 + v*nattr + k; rows of (9 + 3*nattr) floats rounded up
 * to a multiple of 4).  Pack once per scene and data set (again when
 * either changes); vsr_resolve_packed gives the same images, bit for bit,
 * as vsr_resolve on the arrays packed.
 *   vsr_resolve_pack_bytes  bytes of the packed copy (<0 on bad input).
 *   vsr_resolve_pack        xyz, vattr as for vsr_resolve -> packed. */
int64_t vsr_resolve_pack_bytes(int64_t ntri, int32_t nattr);
int vsr_resolve_pack(const float* xyz, const float* vattr, int64_t ntri, int32_t nattr, void* packed,
                     int64_t packed_bytes, void* stream);
int vsr_resolve_packed(const vsr_view* v, int32_t fmt, const void* map, const void* packed, int64_t ntri,
                       int32_t nattr, const uint32_t* tri_id, uint32_t flags, float* bary, float* attr, void* stream);

/* ------------------------------------------------------------- batches */

/* One view of a batch (host memory).  setup/ntri name a resident scene
 * prepared by vsr_setup_tris; the outputs are caller-owned device images. */
typedef struct {
    vsr_view view;
    const void* setup;
    int64_t ntri;
    uint32_t* tri_id;
    float* depth;
} vsr_job;

/* vsr_submit modes */
#define VSR_SUBMIT_BINNED 0 /* all maps, then vsr_bin and vsr_raster work over all jobs (bin_depth used) */
#define VSR_SUBMIT_FUSED 1  /* all maps, then vsr_render work over all jobs (dense, deep scenes)         */

/* Bytes of the workspace vsr_submit needs for these jobs, mode and depth. */
int64_t vsr_submit_bytes(const vsr_job* jobs, int32_t njobs, int32_t fmt, int32_t mode, int32_t bin_depth);

/* Step 5 — many views in one pass: one launch builds every job's map, then
 * one launch per remaining stage covers the pixel blocks of all jobs, so
 * views of different sizes, parameters and scenes share the GPU.  mode
 * VSR_SUBMIT_BINNED bins (bin_depth: 1..2048) and rasterizes; mode
 * VSR_SUBMIT_FUSED runs the fused depth-sliced renderer (bin_depth
 * ignored).  Each job's images are identical, bit for bit, to rendering it
 * alone with vsr_build_map + vsr_bin + vsr_raster or vsr_render at the same
 * fmt.  No host-to-device copy is issued, so the call can be captured in a
 * HIP graph.  Overflowed tiles of the binned mode are counted in the first
 * word of the workspace (vsr_bin_overflow).
 *   jobs       host array of njobs jobs (1..4096).
 *   workspace  device buffer of vsr_submit_bytes(...) bytes holding the job
 *              table, the maps and the bins or list scratch. */
int vsr_submit(const vsr_job* jobs, int32_t njobs, int32_t fmt, int32_t mode, int32_t bin_depth, void* workspace,
               int64_t ws_bytes, void* stream);

/* Instrumented vsr_submit (same work, same images) that also records the
 * caller's HIP events (hipEvent_t passed as void*) on `stream` between its
 * stages: events[0] before the maps, events[1] before the binner (mode
 * VSR_SUBMIT_BINNED) or the fused kernel, events[2] before the rasterizer
 * (binned) or after the fused kernel, events[3] after the last kernel, so
 * that hipEventElapsedTime gives each stage's time on the stream.  nevents
 * must be 4.  For measurement. */
int vsr_submit_timed(const vsr_job* jobs, int32_t njobs, int32_t fmt, int32_t mode, int32_t bin_depth,
                     void* workspace, int64_t ws_bytes, void* const* events, int32_t nevents, void* stream);

/* Graph-friendly batches.  A caller that replays one captured vsr_submit
 * with new view parameters (same sizes, same scenes' triangle counts) writes
 * the job table itself between replays:
 *   vsr_submit_table() fills host_table (vsr_submit_table_bytes(njobs)
 *   bytes) with the table vsr_submit would write for these jobs and this
 *   workspace; the caller copies it to workspace + vsr_submit_table_offset()
 *   on its stream and launches (or replays a capture of) vsr_submit with
 *   mode | VSR_SUBMIT_TABLE_READY, which then reads the table instead of
 *   writing it. */
#define VSR_SUBMIT_TABLE_READY 0x100
/* Binner shape of a binned submit (see VSR_BIN_BLOCKS); neither: automatic
 * over the blocks of all jobs. */
#define VSR_SUBMIT_BIN_BLOCKS 0x200
#define VSR_SUBMIT_BIN_SUPERTILES 0x400
/* 16x16 bin tiles for a binned submit (see VSR_BIN_TILE16). */
#define VSR_SUBMIT_BIN_TILE16 0x800
/* Binned submit: the rasterizer runs as a persistent grid (about as many
 * workgroups as the device holds at once) whose waves take tiles from work
 * counters kept in the workspace header, instead of one workgroup per four
 * tiles or per super-tile.  Same images; only the schedule differs.  No
 * effect on VSR_SUBMIT_FUSED. */
#define VSR_SUBMIT_PERSISTENT 0x1000
int64_t vsr_submit_table_bytes(int32_t njobs);
int64_t vsr_submit_table_offset(void);
int vsr_submit_table(const vsr_job* jobs, int32_t njobs, int32_t fmt, int32_t mode, int32_t bin_depth,
                     const void* workspace, void* host_table, int64_t host_table_bytes);

/* ---------------------------------------------------------- diagnostics */

/* Roofline calibration (measurement only; not part of the method).
 * vsr_calib_copy copies nbytes (a multiple of 16) from src to dst with a
 * streaming kernel (one pass: 2 x nbytes of HBM traffic), to measure the
 * attainable HBM bandwidth.  vsr_calib_fma runs nthreads (a multiple of
 * 256) threads of 8 independent FP32 FMA chains of iters rounds each
 * (nthreads x 8 x iters lane-FMAs) and writes one float per thread to
 * out[nthreads], to measure the attainable non-packed FP32 VALU rate. */
int vsr_calib_copy(const void* src, void* dst, int64_t nbytes, void* stream);
int vsr_calib_fma(float* out, int64_t nthreads, int32_t iters, void* stream);

/* Host call after the stream has synchronised: number of overflowed tiles
 * recorded in a bin buffer (or submit workspace).  Reads device memory with
 * a blocking copy.  Returns VSR_OK or an error code. */
int vsr_bin_overflow(const void* bins_or_ws, int32_t is_workspace, int64_t* overflowed_tiles);

const char* vsr_strerror(int code);
const char* vsr_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* VSR_H */
