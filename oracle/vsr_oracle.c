/*
 * FP64 reference oracle for visual-sphere perspective-map rasterization.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant with the HIP library and never calls it.
 *
 * Every quantity is computed in double precision straight from the paper's
 * definitions, one pixel and one triangle at a time, with no binning,
 * blocking or reordering:
 *
 *   map      Fober, "Perspective picture from Visual Sphere", section 2
 *            (remark on normalising texture coordinates per angle-of-view
 *            type), 2.1.1 (parameter limits) and 2.1.2 (2D->3D transform).
 *   coverage section 1.1 (dot products of the map vector with the three
 *            normalised edge cross products, min of step) and 1.1.1 (binary
 *            step: 1 iff g > 0).
 *   depth    section 1.1.4 (hard normal N=(A-B)x(C-B); r = A.N / G.N).
 *   resolve  section 1.4 (depth-pass test: the nearest r wins).
 *   lens     sections 2.2.2-2.2.4, 2.2.7-2.2.9 (curved panorama, full
 *            dome, equirectangular, cube, screen array and VR maps) and 2.3
 *            (Brown-Conrady distortion of the Universal map's view
 *            coordinates).
 *   wire     section 1.2 (line step of a segment's great circle limited by
 *            the cap around the segment) for the sides of the triangles.
 *   particle section 1.3 (cap of a sphere seen from O, texture coordinates
 *            on the particle's plane), combined as in section 1.4.
 *   aa       sections 1.1.1 (pixel step with the map's global delta), 1.1.2
 *            (miter mask of the smallest circle) and 1.4 (front-to-back
 *            combination of clipped fragment masks).
 *   fragment section 1.1.4, second half (barycentric vector of the
 *            intersection point from triple products with the hard normal;
 *            vertex data interpolated with it).
 *
 * Readings where the paper is silent or inconsistent (all documented in the
 * design notes):
 *   - R = sqrt(x^2 + l*y^2) as in the 2D->3D equation (the inverse in 2.1.3
 *     uses the same form).
 *   - pixel (i, j) samples texture coordinate ((i+1/2)/W, (j+1/2)/H); camera
 *     frame +x right, +y down (row index), +z forward.
 *   - at R = 0 the factor sin(theta)/R takes its limit.
 *   - for k < 0 a pixel with |sin(k*Omega/2)*R| > 1 has no direction
 *     (invalid, never covered).
 *   - triangle winding is arbitrary: the three edge tests are multiplied by
 *     sigma = sign(det[A,B,C]); det = 0 covers nothing.
 *   - ties in depth go to the lower triangle id; no hit gives id 0xFFFFFFFF
 *     and depth +inf.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_NO_HIT 0xFFFFFFFFu
#define ORC_FLAG_EDGE 1u    /* within the 1e-6 rad band of a competing edge */
#define ORC_FLAG_DEPTH 2u   /* best and second-best depth within 2e-5 rel.  */
#define ORC_FLAG_INVALID 4u /* pixel has no view direction                   */
#define ORC_FLAG_DOMAIN 8u  /* within 1e-6 of the projection's domain edge  */

/* Map generators: the Universal Perspective of section 2.1 (with the
 * Brown-Conrady distortion of section 2.3 when any coefficient is non-zero)
 * and the maps of section 2.2: curved panorama (2.2.2), full dome (2.2.3),
 * equirectangular (2.2.4), cube (2.2.7), multiple-screen array (2.2.8) and
 * virtual reality (2.2.9). */
#define ORC_LENS_UNIVERSAL 0
#define ORC_LENS_EQUIRECT 1
#define ORC_LENS_CUBE 2
#define ORC_LENS_SCREENS 3
#define ORC_LENS_VR 4
#define ORC_LENS_PANORAMA 5
#define ORC_LENS_DOME 6

typedef struct {
    int32_t width, height, aov;
    double k, l, s, omega_deg;
    double rot[9];  /* camera -> world, row-major */
    int32_t lens;   /* ORC_LENS_* */
    int32_t lens_n; /* screen array: number of screens */
    double lp[8];   /* lens parameters, see orc_lens_direction */
} orc_view;

static const double ORC_PI = 3.14159265358979323846;

/* ---------------------------------------------------------------------- */
/* Section 2.1.1: clamp k to [-1,1], l to [0,1], s to [4/5,1] and the angle of
 * view (degrees) to [1, Omega_max] with Omega_max = (k>0 ? 179 : 180) /
 * max(|k|, 1/2). */
void orc_limits(double *k, double *l, double *s, double *omega_deg)
{
    double kk = *k < -1.0 ? -1.0 : (*k > 1.0 ? 1.0 : *k);
    double ll = *l < 0.0 ? 0.0 : (*l > 1.0 ? 1.0 : *l);
    double ss = *s < 0.8 ? 0.8 : (*s > 1.0 ? 1.0 : *s);
    double ak = fabs(kk) > 0.5 ? fabs(kk) : 0.5;
    double om_max = (kk > 0.0 ? 179.0 : 180.0) / ak;
    double om = *omega_deg < 1.0 ? 1.0 : (*omega_deg > om_max ? om_max : *omega_deg);
    *k = kk;
    *l = ll;
    *s = ss;
    *omega_deg = om;
}

/* Section 2, remark on 2D coordinates: centre the texture coordinate
 * (fs, ft) in [0,1]^2 and scale it by the aspect ratio a = W/H according to
 * the angle-of-view type.  aov: 0 horizontal, 1 diagonal, 2 vertical,
 * 3 horizontal 4x3. */
static void view_coord_f(double fs, double ft, int32_t width, int32_t height, int32_t aov, double *x, double *y)
{
    double a = (double)width / (double)height;
    double cx = 2.0 * fs - 1.0, cy = 2.0 * ft - 1.0;
    switch (aov) {
    case 1: { /* diagonal: [a, 1] / sqrt(1 + a^2) */
        double q = sqrt(1.0 + a * a);
        *x = cx * a / q;
        *y = cy / q;
        break;
    }
    case 2: /* vertical: [a, 1] */
        *x = cx * a;
        *y = cy;
        break;
    case 3: /* horizontal 4x3: [a, 1] / (4/3) */
        *x = cx * a / (4.0 / 3.0);
        *y = cy / (4.0 / 3.0);
        break;
    default: /* horizontal: [1, 1/a] */
        *x = cx;
        *y = cy / a;
        break;
    }
}

/* The same for the centre of pixel (i, j): ((i + 1/2)/W, (j + 1/2)/H). */
void orc_view_coord(int32_t i, int32_t j, int32_t width, int32_t height, int32_t aov,
                    double *x, double *y)
{
    view_coord_f((i + 0.5) / (double)width, (j + 0.5) / (double)height, width, height, aov, x, y);
}

/* Section 2.1.2: view coordinates (x, y) -> unit direction in the camera
 * frame.  Parameters must already be limited.  Returns 1 when the pixel has
 * a direction, 0 when it falls outside the projection's domain (then out is
 * the zero vector). */
int orc_direction(double x, double y, double k, double l, double s, double omega_deg,
                  double out[3])
{
    double half = 0.5 * omega_deg * ORC_PI / 180.0; /* Omega/2 in radians */
    double R = sqrt(x * x + l * y * y);
    double theta, sin_over_R;
    double c = l * (1.0 - s) + s; /* anamorphic divisor of the y component */
    if (k > 0.0) {
        theta = atan(tan(k * half) * R) / k;
    } else if (k < 0.0) {
        double q = sin(k * half) * R;
        if (q < -1.0 || q > 1.0) {
            out[0] = out[1] = out[2] = 0.0;
            return 0;
        }
        theta = asin(q) / k;
    } else {
        theta = half * R;
    }
    if (R > 0.0) {
        sin_over_R = sin(theta) / R;
    } else { /* limit of sin(theta(R))/R as R -> 0 */
        if (k > 0.0)
            sin_over_R = tan(k * half) / k;
        else if (k < 0.0)
            sin_over_R = sin(k * half) / k;
        else
            sin_over_R = half;
    }
    double v0 = x * sin_over_R;
    double v1 = y * sin_over_R / c;
    double v2 = cos(theta);
    double n = sqrt(v0 * v0 + v1 * v1 + v2 * v2);
    out[0] = v0 / n;
    out[1] = v1 / n;
    out[2] = v2 / n;
    return 1;
}

static void normalize3(double v[3])
{
    double n = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    v[0] /= n;
    v[1] /= n;
    v[2] /= n;
}

/* Section 2.3 Brown-Conrady distortion of view coordinates (x, y):
 * radial (1 + k1 r^2 + k2 r^4), thin prism (p . f) f and decentering q r^2,
 * with c = (k1, k2, p1, p2, q1, q2). */
static void lens_distort(const double *c, double *x, double *y)
{
    double r2 = *x * *x + *y * *y;
    double radial = 1.0 + c[0] * r2 + c[1] * r2 * r2;
    double prism = c[2] * *x + c[3] * *y;
    double nx = *x * radial + prism * *x + c[4] * r2;
    double ny = *y * radial + prism * *y + c[5] * r2;
    *x = nx;
    *y = ny;
}

/* Camera-frame unit direction of texture coordinate (fs, ft) for the view's
 * map generator; *seg receives the picture segment the coordinate belongs
 * to (cube face, screen, eye; 0 for one-piece maps).  Returns 0 (zero
 * direction) where the generator gives none.  Lens parameters lp[]:
 *   UNIVERSAL  (k1, k2, p1, p2, q1, q2) distortion of the view coordinates
 *              (all zero: none), then section 2.1.2 with the view's k, l, s,
 *              Omega after the section 2.1.1 limits;
 *   EQUIRECT   none: longitude pi(2fs - 1), polar angle pi ft from -y;
 *   CUBE       none: six 90-degree faces side by side, face floor(6 fs);
 *   SCREENS    lp[0] = one screen's horizontal angle of view (degrees),
 *              lens_n screens side by side, each turned about y by its
 *              index times that angle;
 *   VR         lp[0] = vertical angle of view (degrees), lp[1] = IPD d in
 *              screen widths, lp[2], lp[3] = radial coefficients k1, k2;
 *   PANORAMA   lp[0] = horizontal angle of view (degrees) of a cylinder of
 *              unit radius whose height follows from the aspect ratio;
 *   DOME       lp[0] = compression angle (degrees), lp[1] = tilt (degrees),
 *              lp[2] = view position offset (in dome radii): a full-dome
 *              fisheye whose angle from the zenith (+y) grows linearly to
 *              90 degrees + compression at the rim; pixels outside the
 *              inscribed circle have no direction. */
int orc_lens_direction(const orc_view *v, double fs, double ft, double out[3], int32_t *seg)
{
    const double a = (double)v->width / (double)v->height;
    const double *p = v->lp;
    *seg = 0;
    switch (v->lens) {
    case ORC_LENS_EQUIRECT: { /* section 2.2.4, equirectangular */
        double lon = ORC_PI * (2.0 * fs - 1.0), pol = ORC_PI * ft;
        out[0] = sin(lon) * sin(pol);
        out[1] = -cos(pol);
        out[2] = cos(lon) * sin(pol);
        return 1;
    }
    case ORC_LENS_CUBE: { /* section 2.2.7, cube mapping */
        int face = (int)floor(6.0 * fs);
        if (face > 5)
            face = 5;
        if (face < 0)
            face = 0;
        double u[3] = {6.0 * fs - face - 0.5, ft - 0.5, 0.5};
        normalize3(u);
        /* rows of each face's rotation; face 3 (absent from the printed
         * cases) is the identity: the forward face */
        static const double M[6][3][3] = {
            {{0, 0, 1}, {-1, 0, 0}, {0, -1, 0}},  /* +x */
            {{0, 0, -1}, {1, 0, 0}, {0, -1, 0}},  /* -x */
            {{1, 0, 0}, {0, -1, 0}, {0, 0, -1}},  /* -z */
            {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}},    /* +z */
            {{1, 0, 0}, {0, 0, 1}, {0, -1, 0}},   /* +y */
            {{-1, 0, 0}, {0, 0, -1}, {0, -1, 0}}, /* -y */
        };
        for (int r = 0; r < 3; ++r)
            out[r] = M[face][r][0] * u[0] + M[face][r][1] * u[1] + M[face][r][2] * u[2];
        *seg = face;
        return 1;
    }
    case ORC_LENS_SCREENS: { /* section 2.2.8, multiple-screen array */
        int n = v->lens_n < 1 ? 1 : v->lens_n;
        int s = (int)floor(n * fs);
        if (s > n - 1)
            s = n - 1;
        if (s < 0)
            s = 0;
        double om = p[0] * ORC_PI / 180.0;
        double phi = (s + 0.5 * (1 - n)) * om;
        double u[3] = {2.0 * (n * fs - s) - 1.0, (2.0 * ft - 1.0) * n / a, 1.0 / tan(0.5 * om)};
        normalize3(u);
        out[0] = cos(phi) * u[0] + sin(phi) * u[2];
        out[1] = u[1];
        out[2] = -sin(phi) * u[0] + cos(phi) * u[2];
        *seg = s;
        return 1;
    }
    case ORC_LENS_VR: { /* section 2.2.9, virtual reality */
        double eye = fs > 0.5 ? 1.0 : (fs < 0.5 ? -1.0 : 0.0);
        double t = 2.0 * fs;
        double x = (2.0 * (t - floor(t)) - 1.0 + eye * (1.0 - 2.0 * p[1])) * 0.5 * a;
        double y = 2.0 * ft - 1.0;
        double R2 = x * x + y * y, den = 1.0 + p[2] + p[3];
        if (den == 0.0) {
            out[0] = out[1] = out[2] = 0.0;
            return 0;
        }
        double f = (1.0 + p[2] * R2 + p[3] * R2 * R2) / den;
        out[0] = x * f;
        out[1] = y * f;
        out[2] = 1.0 / tan(0.5 * p[0] * ORC_PI / 180.0);
        normalize3(out);
        *seg = eye > 0.0 ? 1 : 0;
        return 1;
    }
    case ORC_LENS_DOME: { /* section 2.2.3, full dome */
        double x = 2.0 * fs - 1.0, y = 1.0 - 2.0 * ft;
        double R = sqrt(x * x + y * y);
        if (R > 1.0) {
            out[0] = out[1] = out[2] = 0.0;
            return 0;
        }
        double span = (p[0] + 90.0) * ORC_PI / 180.0;
        double th = R * span;
        double sr = R > 0.0 ? sin(th) / R : span; /* limit of sin(theta)/R at R = 0 */
        double d[3] = {x * sr, cos(th), y * sr + p[2]};
        normalize3(d);
        /* tilt about x, rows of the printed matrix applied to the row vector */
        double t = p[1] * ORC_PI / 180.0, c = cos(t), s = sin(t);
        out[0] = d[0];
        out[1] = d[1] * c + d[2] * s;
        out[2] = -d[1] * s + d[2] * c;
        return 1;
    }
    case ORC_LENS_PANORAMA: { /* section 2.2.2, curved panorama */
        double om = p[0] * ORC_PI / 180.0;
        double x = om * (fs - 0.5), y = (om / a) * (ft - 0.5);
        out[0] = sin(x);
        out[1] = y;
        out[2] = cos(x);
        normalize3(out);
        return 1;
    }
    default: { /* section 2.1 Universal Perspective */
        double k = v->k, l = v->l, s = v->s, om = v->omega_deg, x, y;
        orc_limits(&k, &l, &s, &om);
        view_coord_f(fs, ft, v->width, v->height, v->aov, &x, &y);
        if (p[0] != 0.0 || p[1] != 0.0 || p[2] != 0.0 || p[3] != 0.0 || p[4] != 0.0 || p[5] != 0.0)
            lens_distort(p, &x, &y);
        return orc_direction(x, y, k, l, s, om, out);
    }
    }
}

/* Camera-frame direction and segment of the centre of pixel (i, j). */
int orc_cam_pixel(const orc_view *v, int32_t i, int32_t j, double cam[3], int32_t *seg)
{
    return orc_lens_direction(v, (i + 0.5) / (double)v->width, (j + 0.5) / (double)v->height, cam, seg);
}

/* Pixel (i, j) of a view -> world-space unit direction (camera direction
 * rotated by view->rot). */
int orc_pixel_direction(const orc_view *v, int32_t i, int32_t j, double g[3])
{
    double cam[3];
    int32_t seg;
    int ok = orc_cam_pixel(v, i, j, cam, &seg);
    for (int r = 0; r < 3; ++r)
        g[r] = v->rot[3 * r + 0] * cam[0] + v->rot[3 * r + 1] * cam[1] + v->rot[3 * r + 2] * cam[2];
    return ok;
}

/* 1 when pixel (i, j) lies within 1e-6 of the edge of the projection's
 * domain (k < 0 and |sin(k*Omega/2)*R| within 1e-6 of 1): there the pixel
 * may have a direction in one precision and none in another. */
int orc_domain_edge(const orc_view *v, int32_t i, int32_t j)
{
    double k = v->k, l = v->l, s = v->s, om = v->omega_deg, x, y;
    orc_limits(&k, &l, &s, &om);
    if (v->lens != ORC_LENS_UNIVERSAL || !(k < 0.0))
        return 0;
    orc_view_coord(i, j, v->width, v->height, v->aov, &x, &y);
    if (v->lp[0] != 0.0 || v->lp[1] != 0.0 || v->lp[2] != 0.0 || v->lp[3] != 0.0 || v->lp[4] != 0.0 ||
        v->lp[5] != 0.0)
        lens_distort(v->lp, &x, &y);
    double q = sin(k * 0.5 * om * ORC_PI / 180.0) * sqrt(x * x + l * y * y);
    return fabs(fabs(q) - 1.0) < 1e-6;
}

/* Whole map: dirs[(j*W+i)*3 + c], valid[j*W+i]. */
void orc_map(const orc_view *v, double *dirs, uint8_t *valid)
{
    for (int32_t j = 0; j < v->height; ++j)
        for (int32_t i = 0; i < v->width; ++i) {
            int64_t p = (int64_t)j * v->width + i;
            valid[p] = (uint8_t)orc_pixel_direction(v, i, j, dirs + 3 * p);
        }
}

/* Section 2.1.3: camera-frame unit vector -> view coordinates (x, y).
 * The paper states it as the reverse of 2.1.2; it is exact when
 * l*(1-s)+s = 1.  Parameters must already be limited. */
void orc_inverse(const double v[3], double k, double l, double s, double omega_deg,
                 double *x, double *y)
{
    double half = 0.5 * omega_deg * ORC_PI / 180.0;
    double theta = acos(v[2] / sqrt(v[0] * v[0] + l * v[1] * v[1] + v[2] * v[2]));
    double R;
    if (k > 0.0)
        R = tan(k * theta) / tan(k * half);
    else if (k < 0.0)
        R = sin(k * theta) / sin(k * half);
    else
        R = theta / half;
    double q = sqrt(v[0] * v[0] + l * v[1] * v[1]);
    double f = q > 0.0 ? R / q : 0.0;
    *x = v[0] * f;
    *y = v[1] * f * (l * (1.0 - s) + s);
}

/* ---------------------------------------------------------------------- */
/* Per-triangle quantities.                                                */

static void cross3(const double a[3], const double b[3], double o[3])
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

static double dot3(const double a[3], const double b[3])
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

typedef struct {
    double n[3][3]; /* sigma * normalised A x B, B x C, C x A (section 1.1)  */
    double N[3];    /* hard normal (A-B) x (C-B) (section 1.1.4)             */
    double d;       /* A . N                                                 */
    int live;       /* 0 when det[A,B,C] = 0: covers nothing                 */
} orc_tri;

static void load_vertex(const float *soa, int64_t ntri, int64_t t, int v, double out[3])
{
    out[0] = (double)soa[(3 * v + 0) * ntri + t];
    out[1] = (double)soa[(3 * v + 1) * ntri + t];
    out[2] = (double)soa[(3 * v + 2) * ntri + t];
}

static void tri_prepare(const float *soa, int64_t ntri, int64_t t, orc_tri *o)
{
    double A[3], B[3], C[3], AB[3], BC[3], CA[3], BxC[3], AmB[3], CmB[3];
    load_vertex(soa, ntri, t, 0, A);
    load_vertex(soa, ntri, t, 1, B);
    load_vertex(soa, ntri, t, 2, C);
    cross3(A, B, AB);
    cross3(B, C, BC);
    cross3(C, A, CA);
    cross3(B, C, BxC);
    double det = dot3(A, BxC);
    for (int r = 0; r < 3; ++r) {
        AmB[r] = A[r] - B[r];
        CmB[r] = C[r] - B[r];
    }
    cross3(AmB, CmB, o->N);
    o->d = dot3(A, o->N);
    o->live = det != 0.0;
    double sigma = det > 0.0 ? 1.0 : -1.0;
    const double *e[3] = {AB, BC, CA};
    for (int i = 0; i < 3; ++i) {
        double len = sqrt(dot3(e[i], e[i]));
        if (len == 0.0)
            o->live = 0;
        for (int r = 0; r < 3; ++r)
            o->n[i][r] = len > 0.0 ? sigma * e[i][r] / len : 0.0;
    }
}

/* Exported for tests: the prepared quantities of triangle t.
 * out[0..8] oriented unit edge normals, out[9..11] N, out[12] d, out[13] live. */
void orc_triangle(const float *soa, int64_t ntri, int64_t t, double out[14])
{
    orc_tri o;
    tri_prepare(soa, ntri, t, &o);
    for (int i = 0; i < 3; ++i)
        for (int r = 0; r < 3; ++r)
            out[3 * i + r] = o.n[i][r];
    out[9] = o.N[0];
    out[10] = o.N[1];
    out[11] = o.N[2];
    out[12] = o.d;
    out[13] = o.live;
}

/* Section 1.1.2: smallest circle around the sphere-projected vertices.
 * Circumcentre from barycentric weights a^2(b^2+c^2-a^2) ...; when a weight
 * is <= 0 the triangle is obtuse there and the midpoint of the opposite edge
 * is used.  out = (S_hat, |S|); |S| is the cosine of the cap's radius. */
void orc_cap(const double A[3], const double B[3], const double C[3], double out[4])
{
    double a[3], b[3], c[3], S[3];
    double la = sqrt(dot3(A, A)), lb = sqrt(dot3(B, B)), lc = sqrt(dot3(C, C));
    for (int r = 0; r < 3; ++r) {
        a[r] = A[r] / la;
        b[r] = B[r] / lb;
        c[r] = C[r] / lc;
    }
    double d_bc[3], d_ca[3], d_ab[3];
    for (int r = 0; r < 3; ++r) {
        d_bc[r] = b[r] - c[r];
        d_ca[r] = c[r] - a[r];
        d_ab[r] = a[r] - b[r];
    }
    double a2 = dot3(d_bc, d_bc), b2 = dot3(d_ca, d_ca), c2 = dot3(d_ab, d_ab);
    double ws = a2 * (b2 + c2 - a2);
    double wt = b2 * (c2 + a2 - b2);
    double wp = c2 * (a2 + b2 - c2);
    if (ws <= 0.0) {
        for (int r = 0; r < 3; ++r) S[r] = 0.5 * (b[r] + c[r]);
    } else if (wt <= 0.0) {
        for (int r = 0; r < 3; ++r) S[r] = 0.5 * (c[r] + a[r]);
    } else if (wp <= 0.0) {
        for (int r = 0; r < 3; ++r) S[r] = 0.5 * (a[r] + b[r]);
    } else {
        double w = ws + wt + wp;
        for (int r = 0; r < 3; ++r) S[r] = (ws * a[r] + wt * b[r] + wp * c[r]) / w;
    }
    double len = sqrt(dot3(S, S));
    out[0] = S[0] / len;
    out[1] = S[1] / len;
    out[2] = S[2] / len;
    out[3] = len;
}

/* ---------------------------------------------------------------------- */
/* Brute-force render: every listed pixel against every triangle.           */

typedef struct {
    const orc_view *v;
    const orc_tri *tris;
    int64_t ntri;
    const int64_t *pix; /* NULL: all pixels in row-major order */
    int64_t npix;
    uint32_t *id;
    double *depth;
    double *depth2;
    uint32_t *cover;
    uint8_t *flags;
    int64_t begin, end; /* first pixel and stride */
} orc_job;

/* sin(1e-6): half-width of the edge band in which FP32 and FP64 coverage may
 * legitimately differ. */
static const double BAND = 9.999999999998333e-07;

static void render_pixel(const orc_job *jb, int64_t q)
{
    int64_t p = jb->pix ? jb->pix[q] : q;
    int32_t i = (int32_t)(p % jb->v->width), j = (int32_t)(p / jb->v->width);
    double g[3];
    int ok = orc_pixel_direction(jb->v, i, j, g);
    uint32_t best_id = ORC_NO_HIT, count = 0;
    double best = INFINITY, second = INFINITY;
    double band_min = INFINITY; /* nearest depth of a triangle in the band */
    int band_any = 0;           /* some band triangle with non-positive r  */
    if (ok) {
        for (int64_t t = 0; t < jb->ntri; ++t) {
            const orc_tri *tr = &jb->tris[t];
            if (!tr->live)
                continue;
            double e0 = dot3(tr->n[0], g), e1 = dot3(tr->n[1], g), e2 = dot3(tr->n[2], g);
            double gn = dot3(g, tr->N);
            double r = tr->d / gn;
            if (e0 > 0.0 && e1 > 0.0 && e2 > 0.0) { /* bstep on all three edges */
                ++count;
                if (r < best || (r == best && (uint32_t)t < best_id)) {
                    second = best;
                    best = r;
                    best_id = (uint32_t)t;
                } else if (r < second) {
                    second = r;
                }
            }
            double m0 = fabs(e0), m1 = fabs(e1), m2 = fabs(e2);
            double mn = m0 < m1 ? (m0 < m2 ? m0 : m2) : (m1 < m2 ? m1 : m2);
            if (mn < BAND && e0 > -BAND && e1 > -BAND && e2 > -BAND) {
                if (r > 0.0 && gn != 0.0) {
                    if (r < band_min)
                        band_min = r;
                } else {
                    band_any = 1;
                }
            }
        }
    }
    uint8_t f = 0;
    if (!ok)
        f |= ORC_FLAG_INVALID;
    if (orc_domain_edge(jb->v, i, j))
        f |= ORC_FLAG_DOMAIN;
    if (band_any || (band_min < INFINITY && (best_id == ORC_NO_HIT || band_min <= best * (1.0 + 1e-5))))
        f |= ORC_FLAG_EDGE;
    if (best_id != ORC_NO_HIT && second < INFINITY && second - best <= 2e-5 * best)
        f |= ORC_FLAG_DEPTH;
    jb->id[q] = best_id;
    if (jb->depth) jb->depth[q] = best;
    if (jb->depth2) jb->depth2[q] = second;
    if (jb->cover) jb->cover[q] = count;
    if (jb->flags) jb->flags[q] = f;
}

static void *render_range(void *arg)
{
    orc_job *jb = (orc_job *)arg;
    for (int64_t q = jb->begin; q < jb->npix; q += jb->end)
        render_pixel(jb, q);
    return NULL;
}

/* Render the listed pixels (pix = NULL: the whole W*H frame, row-major).
 * Outputs are indexed like pix; depth2, cover and flags may be NULL.
 * Returns 0 on success, -1 on allocation failure. */
int orc_render(const orc_view *v, const float *xyz_soa, int64_t ntri, const int64_t *pix,
               int64_t npix, uint32_t *id, double *depth, double *depth2, uint32_t *cover,
               uint8_t *flags, int32_t nthreads)
{
    if (!pix)
        npix = (int64_t)v->width * v->height;
    orc_tri *tris = (orc_tri *)malloc(sizeof(orc_tri) * (size_t)(ntri > 0 ? ntri : 1));
    if (!tris)
        return -1;
    for (int64_t t = 0; t < ntri; ++t)
        tri_prepare(xyz_soa, ntri, t, &tris[t]);
    if (nthreads < 1)
        nthreads = 1;
    if (nthreads > 256)
        nthreads = 256;
    pthread_t th[256];
    orc_job jobs[256];
    /* thread w renders pixels w, w + nthreads, w + 2*nthreads, ... */
    for (int w = 0; w < nthreads; ++w) {
        orc_job jb = {v, tris, ntri, pix, npix, id, depth, depth2, cover, flags, w, nthreads};
        jobs[w] = jb;
    }
    for (int w = 1; w < nthreads; ++w)
        pthread_create(&th[w], NULL, render_range, &jobs[w]);
    render_range(&jobs[0]);
    for (int w = 1; w < nthreads; ++w)
        pthread_join(th[w], NULL);
    free(tris);
    return 0;
}

/* One (pixel, triangle) pair: out[0..2] oriented edge values n_i . g,
 * out[3] r = d / (g . N), out[4] pixel valid. */
void orc_pair(const orc_view *v, const float *xyz_soa, int64_t ntri, int64_t t, int64_t p,
              double out[5])
{
    orc_tri tr;
    double g[3];
    tri_prepare(xyz_soa, ntri, t, &tr);
    int ok = orc_pixel_direction(v, (int32_t)(p % v->width), (int32_t)(p / v->width), g);
    out[0] = dot3(tr.n[0], g);
    out[1] = dot3(tr.n[1], g);
    out[2] = dot3(tr.n[2], g);
    out[3] = tr.d / dot3(g, tr.N);
    out[4] = ok;
}

/* ---------------------------------------------------------------------- */
/* Section 1.1.4, fragment data.  For pixel p and triangle t (its winner),
 * the intersection point P = r G with r = A.N / G.N, the barycentric vector
 *   b_s = ((C-P) x (B-P)) . N / (N . N)
 *   b_t = ((A-P) x (C-P)) . N / (N . N)
 *   b_p = ((B-P) x (A-P)) . N / (N . N)
 * (weights of A, B, C) and the vertex data interpolated with it,
 *   f = b_s A_f + b_t B_f + b_p C_f,
 * the first three components normalised when normalize3 (the normal pass).
 * attr holds [3 vertices][nattr][ntri] floats.  A pixel without direction,
 * t = NO_HIT, a degenerate triangle or G parallel to its plane gives b = 0
 * and f = 0. */
static void fragment_one(const orc_view *v, const float *xyz, int64_t ntri, const float *attr, int32_t nattr,
                         int32_t normalize3, int64_t p, uint32_t t, double b[3], double *f)
{
    b[0] = b[1] = b[2] = 0.0;
    for (int32_t k = 0; k < nattr; ++k)
        f[k] = 0.0;
    double g[3];
    if (t == ORC_NO_HIT || (int64_t)t >= ntri)
        return;
    if (!orc_pixel_direction(v, (int32_t)(p % v->width), (int32_t)(p / v->width), g))
        return;
    double A[3], B[3], C[3], AmB[3], CmB[3], N[3];
    load_vertex(xyz, ntri, t, 0, A);
    load_vertex(xyz, ntri, t, 1, B);
    load_vertex(xyz, ntri, t, 2, C);
    for (int r = 0; r < 3; ++r) {
        AmB[r] = A[r] - B[r];
        CmB[r] = C[r] - B[r];
    }
    cross3(AmB, CmB, N);
    double nn = dot3(N, N), gn = dot3(g, N);
    if (nn == 0.0 || gn == 0.0)
        return;
    double r = dot3(A, N) / gn;
    double Pa[3], Pb[3], Pc[3], x[3];
    for (int q = 0; q < 3; ++q) {
        Pa[q] = A[q] - r * g[q];
        Pb[q] = B[q] - r * g[q];
        Pc[q] = C[q] - r * g[q];
    }
    cross3(Pc, Pb, x);
    b[0] = dot3(x, N) / nn;
    cross3(Pa, Pc, x);
    b[1] = dot3(x, N) / nn;
    cross3(Pb, Pa, x);
    b[2] = dot3(x, N) / nn;
    for (int32_t k = 0; k < nattr; ++k) {
        double fa = attr[(0 * (int64_t)nattr + k) * ntri + t];
        double fb = attr[(1 * (int64_t)nattr + k) * ntri + t];
        double fc = attr[(2 * (int64_t)nattr + k) * ntri + t];
        f[k] = b[0] * fa + b[1] * fb + b[2] * fc;
    }
    if (normalize3 && nattr >= 3) {
        double len = sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
        if (len > 0.0)
            for (int q = 0; q < 3; ++q)
                f[q] /= len;
    }
}

/* Fragment data of the listed pixels (flat indices j*W+i) with winners
 * ids[q]: out_b[3q..3q+2], out_f[nattr*q ..]. */
void orc_fragments(const orc_view *v, const float *xyz, int64_t ntri, const float *attr, int32_t nattr,
                   int32_t normalize3, const int64_t *pix, const uint32_t *ids, int64_t npix, double *out_b,
                   double *out_f)
{
    for (int64_t q = 0; q < npix; ++q)
        fragment_one(v, xyz, ntri, attr, nattr, normalize3, pix[q], ids[q], out_b + 3 * q, out_f + nattr * q);
}

/* ---------------------------------------------------------------------- */
/* Aliasing-free coverage: section 1.1.1 (pixel step with the map's global
 * delta), 1.1.2 (miter mask from the smallest circle) and 1.4 (front-to-back
 * combination of fragment masks).                                          */

/* Camera-frame direction of pixel (i, j) (the map before rotation) if it
 * has one and lies in segment seg0 (the neighbour rule of orc_delta). */
static int cam_neighbour(const orc_view *v, int32_t i, int32_t j, int32_t seg0, double g[3])
{
    int32_t seg;
    if (i < 0 || i >= v->width || j < 0 || j >= v->height)
        return 0;
    return orc_cam_pixel(v, i, j, g, &seg) && seg == seg0;
}

/* Derivative of the camera-frame map along one pixel axis at (i, j):
 * central difference of the two neighbours, one-sided where a neighbour is
 * outside the picture, has no direction or lies in another segment of the
 * picture (another cube face, screen or eye: not adjacent on the sphere),
 * 0 when neither neighbour counts. */
static void map_derivative(const orc_view *v, int32_t i, int32_t j, int32_t seg0, int32_t di, int32_t dj,
                           const double g0[3], double out[3])
{
    double gp[3], gm[3];
    int okp = cam_neighbour(v, i + di, j + dj, seg0, gp);
    int okm = cam_neighbour(v, i - di, j - dj, seg0, gm);
    for (int c = 0; c < 3; ++c) {
        if (okp && okm)
            out[c] = 0.5 * (gp[c] - gm[c]);
        else if (okp)
            out[c] = gp[c] - g0[c];
        else if (okm)
            out[c] = g0[c] - gm[c];
        else
            out[c] = 0.0;
    }
}

/* Section 1.1.1 global delta of pixel (i, j): the reciprocal of the largest
 * component of fwidth(G) = |dG/di| + |dG/dj| of the camera-frame map.
 * 0 for a pixel without direction; +inf when the map does not vary. */
double orc_delta(const orc_view *v, int32_t i, int32_t j)
{
    double g[3], di[3], dj[3];
    int32_t seg;
    if (!orc_cam_pixel(v, i, j, g, &seg))
        return 0.0;
    map_derivative(v, i, j, seg, 1, 0, g, di);
    map_derivative(v, i, j, seg, 0, 1, g, dj);
    double m = 0.0;
    for (int c = 0; c < 3; ++c) {
        double f = fabs(di[c]) + fabs(dj[c]);
        if (f > m)
            m = f;
    }
    return m > 0.0 ? 1.0 / m : INFINITY;
}

/* gpstep of section 1.1.1: clamp(delta * g + 1/2, 0, 1).  With an infinite
 * delta (a picture of one pixel: the map does not vary) it is the binary
 * step, and a value exactly on the edge counts as outside, as the strict
 * binary step does. */
static double gpstep(double g, double delta)
{
    double x = delta * g + 0.5;
    return x > 0.0 ? (x < 1.0 ? x : 1.0) : 0.0;
}

#define ORC_AA_AUX 5

typedef struct {
    double r, m, gn;
    uint32_t id;
} orc_frag;

static int frag_cmp(const void *a, const void *b)
{
    const orc_frag *x = (const orc_frag *)a, *y = (const orc_frag *)b;
    if (x->r != y->r)
        return x->r < y->r ? -1 : 1;
    return x->id < y->id ? -1 : (x->id > y->id ? 1 : 0);
}

typedef struct {
    const orc_view *v;
    const orc_tri *tris;
    const double *caps; /* 4 per triangle: S_hat, |S| (section 1.1.2) */
    int64_t ntri;
    const int64_t *pix;
    int64_t npix;
    double *cov, *depth;
    uint32_t *dom;
    double *aux; /* optional, ORC_AA_AUX per pixel: see orc_aa_render */
    int64_t begin, stride;
} orc_aa_job;

/* Fragment mask of a triangle at direction g (sections 1.1.1-1.1.2): the
 * smallest pixel step over the three edges and the miter circle.  The edge
 * values n_i . g have unit gradient on the sphere at the edge; the miter
 * value S_hat . g - |S| has gradient sin(rho) at the rim (|S| = cos rho), so
 * it is divided by sin(rho) before the global delta scales it.  With the
 * per-fragment derivative of the section's equation the division changes
 * nothing (pstep is scale-free); with the global delta it keeps the miter's
 * slope one pixel wide like the edges'.  A degenerate circle (no finite
 * centre, rho = 0, or a circle plane within 1e-6 of O: the projected
 * vertices on one great circle, to rounding) omits the miter, as the
 * section allows. */
static double aa_mask(const orc_tri *tr, const double *cap, const double g[3], double delta)
{
    double m = 1.0;
    for (int i = 0; i < 3; ++i) {
        double s = gpstep(dot3(tr->n[i], g), delta);
        if (s < m)
            m = s;
    }
    if (isfinite(cap[0]) && isfinite(cap[1]) && isfinite(cap[2]) && isfinite(cap[3]) && cap[3] > 1e-6) {
        double sr2 = 1.0 - cap[3] * cap[3];
        if (sr2 > 0.0) {
            double s = gpstep((dot3(cap, g) - cap[3]) / sqrt(sr2), delta);
            if (s < m)
                m = s;
        }
    }
    return m;
}

static void aa_pixel(const orc_aa_job *jb, int64_t q)
{
    int64_t p = jb->pix ? jb->pix[q] : q;
    int32_t i = (int32_t)(p % jb->v->width), j = (int32_t)(p / jb->v->width);
    double g[3];
    double m_b = 0.0, r_b = 0.0, best = 0.0, second = 0.0, gap = INFINITY;
    double n_near = 0.0, sum_r = 0.0, sum_rg = 0.0;
    uint32_t dom = ORC_NO_HIT;
    if (orc_pixel_direction(jb->v, i, j, g)) {
        double delta = orc_delta(jb->v, i, j);
        int64_t cap_n = 16, n = 0;
        orc_frag *fr = (orc_frag *)malloc(sizeof(orc_frag) * (size_t)cap_n);
        for (int64_t t = 0; fr && t < jb->ntri; ++t) {
            const orc_tri *tr = &jb->tris[t];
            if (!tr->live)
                continue;
            double m = aa_mask(tr, jb->caps + 4 * t, g, delta);
            double gn = dot3(g, tr->N);
            if (!(m > 0.0) || gn == 0.0)
                continue;
            double r = tr->d / gn;
            if (!(r > 0.0))
                continue;
            if (n == cap_n) {
                cap_n *= 2;
                orc_frag *nf = (orc_frag *)realloc(fr, sizeof(orc_frag) * (size_t)cap_n);
                if (!nf) {
                    free(fr);
                    fr = NULL;
                    break;
                }
                fr = nf;
            }
            fr[n].r = r;
            fr[n].m = m;
            fr[n].gn = fabs(gn) / sqrt(dot3(tr->N, tr->N));
            fr[n].id = (uint32_t)t;
            ++n;
        }
        if (fr) {
            qsort(fr, (size_t)n, sizeof(orc_frag), frag_cmp);
            /* section 1.4: front to back, each mask clipped by what is
             * already covered, data weighted by the clipped mask */
            int64_t k = 0;
            for (; k < n && m_b < 1.0; ++k) {
                double mfc = fr[k].m < 1.0 - m_b ? fr[k].m : 1.0 - m_b;
                m_b += mfc;
                r_b += mfc * fr[k].r;
                if (mfc > best) {
                    second = best;
                    best = mfc;
                    dom = fr[k].id;
                } else if (mfc > second) {
                    second = mfc;
                }
            }
            /* conditioning over the fragments taken and the first one left
             * out: smallest relative depth step (below rounding their order
             * is arbitrary), their number, sum of depths and of depth over
             * the cosine between ray and plane normal */
            for (int64_t f = 0; f <= k && f < n; ++f) {
                if (f > 0) {
                    double step = (fr[f].r - fr[f - 1].r) / fr[f].r;
                    if (step < gap)
                        gap = step;
                }
                n_near += 1.0;
                sum_r += fr[f].r;
                sum_rg += fr[f].r / fr[f].gn;
            }
            free(fr);
        }
    }
    jb->cov[q] = m_b;
    jb->depth[q] = r_b;
    jb->dom[q] = dom;
    if (jb->aux) {
        double *a = jb->aux + ORC_AA_AUX * q;
        a[0] = best - second;
        a[1] = gap;
        a[2] = n_near;
        a[3] = sum_r;
        a[4] = sum_rg;
    }
}

static void *aa_range(void *arg)
{
    orc_aa_job *jb = (orc_aa_job *)arg;
    for (int64_t q = jb->begin; q < jb->npix; q += jb->stride)
        aa_pixel(jb, q);
    return NULL;
}

/* Anti-aliased render of the listed pixels (pix = NULL: whole frame):
 * coverage m in [0, 1], depth pass sum(m_fc * r) and the id with the largest
 * clipped mask (NO_HIT when nothing covers; on equal clipped masks the
 * nearer fragment).  aux (optional, ORC_AA_AUX per pixel) receives, for a
 * tolerance model of a lower-precision implementation: the margin of the
 * largest clipped mask over the second largest; the smallest relative depth
 * step between consecutive fragments among those taken and the first one
 * left out (+inf if none; where either is at rounding level another
 * dominant id is as correct); the number of those fragments, the sum of
 * their depths r, and the sum of r / cos(ray, plane normal).  Returns -1 on
 * allocation failure. */
int orc_aa_render(const orc_view *v, const float *xyz_soa, int64_t ntri, const int64_t *pix, int64_t npix,
                  double *cov, double *depth, uint32_t *dom, double *aux, int32_t nthreads)
{
    if (!pix)
        npix = (int64_t)v->width * v->height;
    orc_tri *tris = (orc_tri *)malloc(sizeof(orc_tri) * (size_t)(ntri > 0 ? ntri : 1));
    double *caps = (double *)malloc(sizeof(double) * 4 * (size_t)(ntri > 0 ? ntri : 1));
    if (!tris || !caps) {
        free(tris);
        free(caps);
        return -1;
    }
    for (int64_t t = 0; t < ntri; ++t) {
        double A[3], B[3], C[3];
        tri_prepare(xyz_soa, ntri, t, &tris[t]);
        load_vertex(xyz_soa, ntri, t, 0, A);
        load_vertex(xyz_soa, ntri, t, 1, B);
        load_vertex(xyz_soa, ntri, t, 2, C);
        if (tris[t].live)
            orc_cap(A, B, C, caps + 4 * t);
    }
    if (nthreads < 1)
        nthreads = 1;
    if (nthreads > 256)
        nthreads = 256;
    pthread_t th[256];
    orc_aa_job jobs[256];
    for (int w = 0; w < nthreads; ++w) {
        orc_aa_job jb = {v, tris, caps, ntri, pix, npix, cov, depth, dom, aux, w, nthreads};
        jobs[w] = jb;
    }
    for (int w = 1; w < nthreads; ++w)
        pthread_create(&th[w], NULL, aa_range, &jobs[w]);
    aa_range(&jobs[0]);
    for (int w = 1; w < nthreads; ++w)
        pthread_join(th[w], NULL);
    free(tris);
    free(caps);
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Wire-frame line segments (section 1.2) and procedural particles
 * (section 1.3), aliasing-free, with the global delta of section 1.1.1.    */

typedef struct {
    void (*fn)(void *ctx, int64_t q);
    void *ctx;
    int64_t n, begin, stride;
} orc_par;

static void *par_range(void *arg)
{
    orc_par *p = (orc_par *)arg;
    for (int64_t q = p->begin; q < p->n; q += p->stride)
        p->fn(p->ctx, q);
    return NULL;
}

static void par_for(int64_t n, int32_t nthreads, void (*fn)(void *, int64_t), void *ctx)
{
    if (nthreads < 1)
        nthreads = 1;
    if (nthreads > 256)
        nthreads = 256;
    pthread_t th[256];
    orc_par jobs[256];
    for (int w = 0; w < nthreads; ++w) {
        orc_par p = {fn, ctx, n, w, nthreads};
        jobs[w] = p;
    }
    for (int w = 1; w < nthreads; ++w)
        pthread_create(&th[w], NULL, par_range, &jobs[w]);
    par_range(&jobs[0]);
    for (int w = 1; w < nthreads; ++w)
        pthread_join(th[w], NULL);
}

/* One line segment P->Q on the sphere: the unit normal of its great circle
 * and the cap around it (centre L_hat = normalised mean of the unit end
 * points, cos of the radius |L|).  Returns 0 when the great circle is
 * undefined (P and Q on one line through O). */
typedef struct {
    double n[3], L[3], cos_r, sin_r;
} orc_seg;

static int seg_prepare(const double P[3], const double Q[3], orc_seg *s)
{
    double p[3], q[3], c[3];
    double lp = sqrt(dot3(P, P)), lq = sqrt(dot3(Q, Q));
    if (!(lp > 0.0) || !(lq > 0.0))
        return 0;
    for (int r = 0; r < 3; ++r) {
        p[r] = P[r] / lp;
        q[r] = Q[r] / lq;
    }
    cross3(p, q, c);
    double ln = sqrt(dot3(c, c));
    if (!(ln > 0.0))
        return 0;
    double L[3] = {0.5 * (p[0] + q[0]), 0.5 * (p[1] + q[1]), 0.5 * (p[2] + q[2])};
    double ll = sqrt(dot3(L, L));
    if (!(ll > 0.0))
        return 0;
    for (int r = 0; r < 3; ++r) {
        s->n[r] = c[r] / ln;
        s->L[r] = L[r] / ll;
    }
    s->cos_r = ll;
    s->sin_r = sqrt(1.0 - ll * ll > 0.0 ? 1.0 - ll * ll : 0.0);
    return 1;
}

/* Line mask of a segment at direction g: the pixel-smooth line step of the
 * great circle, 1 - min(|n.g| delta, 1), limited by the pixel step of the
 * cap around the segment (its value divided by sin of the radius, as for
 * the miter mask). */
static double seg_mask(const orc_seg *s, const double g[3], double delta)
{
    double h = fabs(dot3(s->n, g)) * delta;
    h = h < 1.0 ? 1.0 - h : 0.0;
    if (!(h > 0.0))
        return 0.0;
    if (s->sin_r > 0.0) {
        double c = gpstep((dot3(s->L, g) - s->cos_r) / s->sin_r, delta);
        if (c < h)
            h = c;
    }
    return h;
}

typedef struct {
    const orc_view *v;
    const float *xyz;
    int64_t ntri;
    const orc_seg *segs; /* 3 per triangle */
    const uint8_t *seg_ok;
    const int64_t *pix;
    double *cov;
    uint32_t *dom;
    double *second; /* optional: second largest value among other triangles */
} orc_wire_job;

static void wire_pixel(void *ctx, int64_t q)
{
    const orc_wire_job *jb = (const orc_wire_job *)ctx;
    int64_t p = jb->pix ? jb->pix[q] : q;
    int32_t i = (int32_t)(p % jb->v->width), j = (int32_t)(p / jb->v->width);
    double g[3], best = 0.0, second = 0.0;
    uint32_t dom = ORC_NO_HIT;
    if (orc_pixel_direction(jb->v, i, j, g)) {
        double delta = orc_delta(jb->v, i, j);
        for (int64_t t = 0; t < jb->ntri; ++t) {
            double mt = 0.0;
            for (int e = 0; e < 3; ++e)
                if (jb->seg_ok[3 * t + e]) {
                    double m = seg_mask(&jb->segs[3 * t + e], g, delta);
                    if (m > mt)
                        mt = m;
                }
            if (mt > best) {
                second = best;
                best = mt;
                dom = (uint32_t)t;
            } else if (mt > second) {
                second = mt;
            }
        }
    }
    jb->cov[q] = best;
    jb->dom[q] = dom;
    if (jb->second)
        jb->second[q] = second;
}

/* Wire frame of the live triangles' sides (segments AB, BC, CA): per pixel
 * the largest line mask over all sides and the triangle it belongs to (ties:
 * the lower id; NO_HIT when every mask is 0); `second` (optional) receives
 * the largest mask of any other triangle.  Returns -1 on allocation
 * failure. */
int orc_wireframe(const orc_view *v, const float *xyz_soa, int64_t ntri, const int64_t *pix, int64_t npix,
                  double *cov, uint32_t *dom, double *second, int32_t nthreads)
{
    if (!pix)
        npix = (int64_t)v->width * v->height;
    size_t m = (size_t)(ntri > 0 ? ntri : 1);
    orc_seg *segs = (orc_seg *)malloc(sizeof(orc_seg) * 3 * m);
    uint8_t *ok = (uint8_t *)malloc(3 * m);
    if (!segs || !ok) {
        free(segs);
        free(ok);
        return -1;
    }
    for (int64_t t = 0; t < ntri; ++t) {
        double V[3][3];
        orc_tri tr;
        tri_prepare(xyz_soa, ntri, t, &tr);
        for (int c = 0; c < 3; ++c)
            load_vertex(xyz_soa, ntri, t, c, V[c]);
        for (int e = 0; e < 3; ++e)
            ok[3 * t + e] = (uint8_t)(tr.live && seg_prepare(V[e], V[(e + 1) % 3], &segs[3 * t + e]));
    }
    orc_wire_job jb = {v, xyz_soa, ntri, segs, ok, pix, cov, dom, second};
    par_for(npix, nthreads, wire_pixel, &jb);
    free(segs);
    free(ok);
    return 0;
}

/* Particles: position P (from O) and radius r, P.P > r^2 > 0. */
typedef struct {
    double P[3], dist, cos_r, sin_r, X[3], Y[3], scale;
    int live;
} orc_part;

static void part_prepare(const float *pr, int64_t n, int64_t k, orc_part *o)
{
    double P[3] = {pr[0 * n + k], pr[1 * n + k], pr[2 * n + k]}, r = pr[3 * n + k];
    double d = sqrt(dot3(P, P));
    o->live = r > 0.0 && d > r;
    if (!o->live)
        return;
    for (int c = 0; c < 3; ++c)
        o->P[c] = P[c] / d;
    o->dist = d;
    o->sin_r = r / d;
    o->cos_r = sqrt(1.0 - o->sin_r * o->sin_r);
    /* texture axes: X = |(P_z, 0, -P_x)| (x axis when P is vertical), Y = X x P_hat */
    double xl = sqrt(P[2] * P[2] + P[0] * P[0]);
    if (xl > 0.0) {
        o->X[0] = P[2] / xl;
        o->X[1] = 0.0;
        o->X[2] = -P[0] / xl;
    } else {
        o->X[0] = 1.0;
        o->X[1] = 0.0;
        o->X[2] = 0.0;
    }
    cross3(o->X, o->P, o->Y);
    o->scale = d / (2.0 * r);
}

typedef struct {
    const orc_view *v;
    const orc_part *parts;
    int64_t n;
    const int64_t *pix;
    double *cov, *depth, *uv;
    uint32_t *dom;
    double *aux;
} orc_part_job;

typedef struct {
    double r, m, u, w;
    uint32_t id;
} orc_pfrag;

static int pfrag_cmp(const void *a, const void *b)
{
    const orc_pfrag *x = (const orc_pfrag *)a, *y = (const orc_pfrag *)b;
    if (x->r != y->r)
        return x->r < y->r ? -1 : 1;
    return x->id < y->id ? -1 : (x->id > y->id ? 1 : 0);
}

static void part_pixel(void *ctx, int64_t q)
{
    const orc_part_job *jb = (const orc_part_job *)ctx;
    int64_t p = jb->pix ? jb->pix[q] : q;
    int32_t i = (int32_t)(p % jb->v->width), j = (int32_t)(p / jb->v->width);
    double g[3], m_b = 0.0, r_b = 0.0, u_b = 0.0, w_b = 0.0, best = 0.0, second = 0.0, gap = INFINITY;
    double n_near = 0.0, sum_r = 0.0;
    uint32_t dom = ORC_NO_HIT;
    if (orc_pixel_direction(jb->v, i, j, g)) {
        double delta = orc_delta(jb->v, i, j);
        int64_t cap_n = 16, n = 0;
        orc_pfrag *fr = (orc_pfrag *)malloc(sizeof(orc_pfrag) * (size_t)cap_n);
        for (int64_t k = 0; fr && k < jb->n; ++k) {
            const orc_part *pt = &jb->parts[k];
            if (!pt->live)
                continue;
            double gp = dot3(g, pt->P);
            double m = gpstep((gp - pt->cos_r) / pt->sin_r, delta);
            if (!(m > 0.0) || !(gp > 0.0))
                continue;
            if (n == cap_n) {
                cap_n *= 2;
                orc_pfrag *nf = (orc_pfrag *)realloc(fr, sizeof(orc_pfrag) * (size_t)cap_n);
                if (!nf) {
                    free(fr);
                    fr = NULL;
                    break;
                }
                fr = nf;
            }
            fr[n].r = pt->dist / gp; /* where the ray meets the particle's plane */
            fr[n].m = m;
            fr[n].u = dot3(g, pt->X) * pt->scale + 0.5;
            fr[n].w = dot3(g, pt->Y) * pt->scale + 0.5;
            fr[n].id = (uint32_t)k;
            ++n;
        }
        if (fr) {
            qsort(fr, (size_t)n, sizeof(orc_pfrag), pfrag_cmp);
            int64_t k = 0;
            for (; k < n && m_b < 1.0; ++k) { /* section 1.4, texture coordinates as a pass too */
                double mfc = fr[k].m < 1.0 - m_b ? fr[k].m : 1.0 - m_b;
                m_b += mfc;
                r_b += mfc * fr[k].r;
                u_b += mfc * fr[k].u;
                w_b += mfc * fr[k].w;
                if (mfc > best) {
                    second = best;
                    best = mfc;
                    dom = fr[k].id;
                } else if (mfc > second) {
                    second = mfc;
                }
            }
            for (int64_t f = 0; f <= k && f < n; ++f) {
                if (f > 0) {
                    double step = (fr[f].r - fr[f - 1].r) / fr[f].r;
                    if (step < gap)
                        gap = step;
                }
                n_near += 1.0;
                sum_r += fr[f].r;
            }
            free(fr);
        }
    }
    jb->cov[q] = m_b;
    jb->depth[q] = r_b;
    jb->uv[2 * q] = u_b;
    jb->uv[2 * q + 1] = w_b;
    jb->dom[q] = dom;
    if (jb->aux) {
        double *a = jb->aux + 4 * q;
        a[0] = best - second;
        a[1] = gap;
        a[2] = n_near;
        a[3] = sum_r;
    }
}

/* Particles (pr = float[4][n]: x, y, z, radius), section 1.3 mask with the
 * pixel step of section 1.1.1 (the cap value divided by sin of its radius,
 * like the miter mask), combined front to back by the depth where the ray
 * meets the particle's plane (through P, normal P_hat) as in section 1.4:
 * coverage, depth pass, texture-coordinate pass (2 per pixel) and dominant
 * id.  aux (optional, 4 per pixel): share margin, smallest relative depth
 * step, fragments taken + 1, their summed depth.  Particles with r <= 0 or
 * the camera inside are skipped.  Returns -1 on allocation failure. */
int orc_particles(const orc_view *v, const float *pr, int64_t n, const int64_t *pix, int64_t npix, double *cov,
                  double *depth, double *uv, uint32_t *dom, double *aux, int32_t nthreads)
{
    if (!pix)
        npix = (int64_t)v->width * v->height;
    orc_part *parts = (orc_part *)malloc(sizeof(orc_part) * (size_t)(n > 0 ? n : 1));
    if (!parts)
        return -1;
    for (int64_t k = 0; k < n; ++k)
        part_prepare(pr, n, k, &parts[k]);
    orc_part_job jb = {v, parts, n, pix, cov, depth, uv, dom, aux};
    par_for(npix, nthreads, part_pixel, &jb);
    free(parts);
    return 0;
}
