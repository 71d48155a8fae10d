/*
 * FP64 CPU oracle for the phase-space-tessellation column-density projection.
 *
 * TEST INFRASTRUCTURE ONLY.  This is the slow, plain reference that the GPU
 * library is checked against.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it.  It shares no code, header,
 * table or helper with the GPU library, and the GPU library never calls it.
 *
 * What it computes (point sampling at pixel centres):
 *
 *   I(ix, iy) = sum over lattice cubes, sum over the six tetrahedra T of the
 *               cube, of q(T) * length(ray(ix, iy) inside T),
 *   q(T) = rho(T)^p,  rho(T) = m / |V(T)|,  p = qpow in {0, 1, 2}
 *
 * which is the line-of-sight projection of Eq. Eqn:TetProjection with a
 * constant per-tetrahedron value q: p = 1 is the column density (q = rho_loc
 * of Eq. Eqn-rho_loc, with the overlap sum of Eq. Eqn-rho_tot_b); p = 0 and
 * p = 2 are the density projections of Eq. Eqn-column-density with g = 1 (the
 * path length summed over streams, the line-of-sight integral of the stream
 * count) and g = rho^2.  The
 * cell-projection section (Eq. Eqn:TetSum) evaluates the same sum with a
 * camera-distance split; the oracle uses the plain per-ray clip instead.
 *
 * Steps, in the paper's order and notation:
 *  1. Tracer id -> lattice vertex (i, j, k) with id = i + d0 (j + d1 k)
 *     (Eq. Eqn:ID).  Cube (i, j, k) has corners n = a + 2b + 4c at
 *     (i + a, j + b, k + c), taken modulo the lattice when periodic.
 *  2. Periodic unwrap: every corner is moved to the periodic image nearest
 *     to corner 0 of its cube, one component at a time; an offset of exactly
 *     half the box is taken in the positive direction, i.e. the offset lies
 *     in (-L/2, L/2].
 *  3. Six tetrahedra per cube from the connectivity table of the
 *     data-storage section: {1,0,2,4} {3,1,2,4} {3,5,1,4} {3,6,5,4}
 *     {3,2,6,4} {3,7,5,6}.
 *  4. Signed volume V = (v1 - v0) . ((v2 - v0) x (v3 - v0)) / 6
 *     (Eq. Eqn:TetVolume); V == 0 is skipped and counted; density
 *     rho = m / |V| with tetrahedron mass m = M / (6 * cubes).
 *  5. Orthographic view: y = R (x - c), rows of R = (screen u, screen v,
 *     view direction).  Pixel centres at u = -Su/2 + (ix + 1/2) Su / W.
 *  6. Each pixel ray {(pu, pv, t)} is clipped against the four outward face
 *     planes n . y <= h; dl = max(0, t_exit - t_entry).  With a depth slab
 *     [s0, s1] the chord is clipped to it as well (the slab-clamped front and
 *     back fragments of the resampling section, Eqs. Eqn:ResFF, Eqn:ResBF).  A face parallel to
 *     the ray (n_d == 0) excludes the ray when h - n_u pu - n_v pv < 0; on
 *     the plane itself the ray is kept iff n_u < 0, or n_u == 0 and n_v < 0
 *     (a half-open rule, so exactly one of two face-sharing tets keeps it).
 *  7. I += q * dl with Neumaier-compensated FP64 sums.  With image wrap
 *     the pixel index is taken modulo (W, H); otherwise pixels outside the
 *     window are dropped.
 *  Perspective view (the camera point c of Eq. Eqn:TetSum, the camera inside
 *  the volume of the large-scale figure): c is the camera, R its axes, and
 *  the pixel at (pu, pv) on the plane at unit distance along the view
 *  direction sees the half-line {s (pu, pv, 1) : s >= 0} in view space; a face
 *  with n . d == 0 excludes it when h < 0 (and on the plane, h == 0, by the
 *  half-open rule above); dl = |(pu, pv, 1)| (s_exit - max(s_entry, 0)).  No
 *  wrap and no slab.
 *  Centroids and the near/far hybrid under the perspective camera (the
 *  centroid section's billboards; the large-scale figure's hybrid): a
 *  billboard faces the view direction at T's centroid y_c (camera frame) and
 *  adds q |V| W(r, h) to the pixel whose ray crosses its plane at distance
 *  r = z_c |(pu, pv) - (x_c, y_c) / z_c| from y_c, h = |V|^(1/3), W the 2D
 *  cubic spline of orc_splat_image; only centroids in front of the camera
 *  (z_c > 0) are drawn.  Hybrid: T within lod_radius of the camera (|y_c|
 *  <= lod_radius) is clipped exactly, the rest are billboards.
 *
 * Determinism: region mode assigns every image row band to one thread and
 * visits tetrahedra in id order, so results do not depend on the thread
 * count.  Pixel-sample mode keeps per-thread partial sums and adds them in
 * thread order (deterministic for a fixed thread count).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define ORC_OK 0
#define ORC_EINVAL -1
#define ORC_ENOMEM -2

typedef struct {
    int32_t dims[3];      /* vertices per axis */
    double box[3];        /* periodic box lengths */
    int32_t periodic;     /* 1: d0*d1*d2 cubes with wrap; 0: (d0-1)(d1-1)(d2-1) */
    double total_mass;    /* M */
    double rot[9];        /* row-major view rotation */
    double center[3];     /* world point at the image centre */
    double extent[2];     /* window size (u, v) */
    int32_t width, height;
    int32_t wrap;         /* pixel index modulo (W, H) */
    int32_t qpow;         /* projected value q = rho^qpow, qpow in {0, 1, 2} */
    int32_t slab;         /* 1: only the depths t in [slab_t[0], slab_t[1]] count */
    double slab_t[2];     /* depth t = third view coordinate, R (x - c) */
    int32_t perspective;  /* 1: rays from the camera c (step 5 otherwise) */
    int32_t method;       /* perspective: 0 exact, 1 centroid billboards, 2 hybrid */
    double lod_radius;    /* hybrid: exact within this distance of the camera */
} orc_problem;

typedef struct {
    int64_t tets;         /* tetrahedra with V != 0 */
    int64_t zero_volume;  /* skipped, V == 0 */
    int64_t inverted;     /* V > 0 (the undisplaced lattice has V < 0) */
    int64_t fragments;    /* (pixel, tet) pairs with dl > 0 inside the target */
} orc_stats;

static const int TET_TABLE[6][4] = {
    {1, 0, 2, 4}, {3, 1, 2, 4}, {3, 5, 1, 4}, {3, 6, 5, 4}, {3, 2, 6, 4}, {3, 7, 5, 6}};

typedef struct {
    int persp;            /* rays from the camera at the view-space origin */
    int splat;            /* a billboard (perspective centroids): q = q |V|, */
    double uc, vc, zc, hh;  /* window centre, depth, kernel size */
    double q;             /* projected value rho^qpow */
    double s0, s1;        /* depth slab (-inf, inf without one) */
    double n[4][3];       /* outward normals in view space */
    double h[4];          /* plane offsets, n . y <= h inside */
    int64_t ix0, ix1, iy0, iy1;  /* candidate pixel range (inclusive, unwrapped) */
} orc_tet;

/* ---------------------------------------------------------------- helpers */
static inline void neu_add(double *s, double *c, double x) {
    double t = *s + x;
    if (fabs(*s) >= fabs(x))
        *c += (*s - t) + x;
    else
        *c += (x - t) + *s;
    *s = t;
}

static inline int64_t imod(int64_t a, int64_t m) {
    int64_t r = a % m;
    return r < 0 ? r + m : r;
}

static int64_t n_cubes(const orc_problem *P) {
    int64_t c[3];
    for (int a = 0; a < 3; ++a) c[a] = P->periodic ? P->dims[a] : P->dims[a] - 1;
    return c[0] * c[1] * c[2];
}

static int check_problem(const orc_problem *P) {
    if (!P) return ORC_EINVAL;
    for (int a = 0; a < 3; ++a) {
        if (P->dims[a] < 2) return ORC_EINVAL;
        if (!(P->box[a] > 0)) return ORC_EINVAL;
    }
    if (P->width < 1 || P->height < 1) return ORC_EINVAL;
    if (!(P->extent[0] > 0) || !(P->extent[1] > 0)) return ORC_EINVAL;
    if (!(P->total_mass > 0)) return ORC_EINVAL;
    if (P->qpow < 0 || P->qpow > 2) return ORC_EINVAL;
    if (P->slab && !(P->slab_t[0] < P->slab_t[1])) return ORC_EINVAL;
    if (P->perspective && (P->wrap || P->slab)) return ORC_EINVAL;
    if (P->method < 0 || P->method > 2 || (P->method && !P->perspective)) return ORC_EINVAL;
    if (P->method == 2 && !(P->lod_radius >= 0.0 && isfinite(P->lod_radius))) return ORC_EINVAL;
    return ORC_OK;
}

/* Corner positions (world, unwrapped to the periodic image nearest corner 0)
 * of lattice cube `cube` (cube id = i + c0 (j + c1 k) over the cube grid). */
static void cube_corners(const orc_problem *P, const float *x, const float *y,
                         const float *z, int64_t cube, double X[8][3]) {
    int64_t c0 = P->periodic ? P->dims[0] : P->dims[0] - 1;
    int64_t c1 = P->periodic ? P->dims[1] : P->dims[1] - 1;
    int64_t i = cube % c0, j = (cube / c0) % c1, k = cube / (c0 * c1);
    for (int n = 0; n < 8; ++n) {
        int64_t ii = i + (n & 1), jj = j + ((n >> 1) & 1), kk = k + ((n >> 2) & 1);
        if (P->periodic) {
            ii = imod(ii, P->dims[0]);
            jj = imod(jj, P->dims[1]);
            kk = imod(kk, P->dims[2]);
        }
        int64_t id = ii + (int64_t)P->dims[0] * (jj + (int64_t)P->dims[1] * kk);
        X[n][0] = (double)x[id];
        X[n][1] = (double)y[id];
        X[n][2] = (double)z[id];
    }
    if (P->periodic) {
        for (int n = 1; n < 8; ++n)
            for (int a = 0; a < 3; ++a) {
                double e = X[n][a] - X[0][a];
                e -= P->box[a] * ceil(e / P->box[a] - 0.5);
                X[n][a] = X[0][a] + e;
            }
    }
}

static double signed_volume(const double v[4][3]) {
    double a[3], b[3], c[3];
    for (int q = 0; q < 3; ++q) {
        a[q] = v[1][q] - v[0][q];
        b[q] = v[2][q] - v[0][q];
        c[q] = v[3][q] - v[0][q];
    }
    double cx = b[1] * c[2] - b[2] * c[1];
    double cy = b[2] * c[0] - b[0] * c[2];
    double cz = b[0] * c[1] - b[1] * c[0];
    return (a[0] * cx + a[1] * cy + a[2] * cz) / 6.0;
}

/* Build the view-space clip description of one tetrahedron.  Returns 0 when
 * the tetrahedron is skipped (V == 0), 1 otherwise; *V receives the volume. */
static int tet_setup(const orc_problem *P, const double v[4][3], double mass,
                     orc_tet *t, double *V) {
    *V = signed_volume(v);
    if (*V == 0.0) return 0;
    const double rho = mass / fabs(*V);
    t->q = P->qpow == 0 ? 1.0 : (P->qpow == 1 ? rho : rho * rho);
    t->s0 = P->slab ? P->slab_t[0] : -INFINITY;
    t->s1 = P->slab ? P->slab_t[1] : INFINITY;
    double yv[4][3];
    for (int m = 0; m < 4; ++m) {
        double d[3] = {v[m][0] - P->center[0], v[m][1] - P->center[1], v[m][2] - P->center[2]};
        for (int r = 0; r < 3; ++r)
            yv[m][r] = P->rot[3 * r] * d[0] + P->rot[3 * r + 1] * d[1] + P->rot[3 * r + 2] * d[2];
    }
    for (int a = 0; a < 4; ++a) {
        int b = (a + 1) & 3, c = (a + 2) & 3, d = (a + 3) & 3;
        double e1[3], e2[3], ea[3];
        for (int q = 0; q < 3; ++q) {
            e1[q] = yv[c][q] - yv[b][q];
            e2[q] = yv[d][q] - yv[b][q];
            ea[q] = yv[a][q] - yv[b][q];
        }
        double nn[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                        e1[0] * e2[1] - e1[1] * e2[0]};
        double side = nn[0] * ea[0] + nn[1] * ea[1] + nn[2] * ea[2];
        if (side > 0) { nn[0] = -nn[0]; nn[1] = -nn[1]; nn[2] = -nn[2]; }
        t->n[a][0] = nn[0]; t->n[a][1] = nn[1]; t->n[a][2] = nn[2];
        t->h[a] = nn[0] * yv[b][0] + nn[1] * yv[b][1] + nn[2] * yv[b][2];
    }
    t->persp = P->perspective;
    t->splat = 0;
    if (P->perspective && P->method != 0) {
        double yc[3] = {0, 0, 0};
        for (int m = 0; m < 4; ++m)
            for (int r = 0; r < 3; ++r) yc[r] += 0.25 * yv[m][r];
        const double dist = sqrt(yc[0] * yc[0] + yc[1] * yc[1] + yc[2] * yc[2]);
        if (P->method == 1 || dist > P->lod_radius) {
            t->splat = 1;
            t->hh = cbrt(fabs(*V));
            t->q *= fabs(*V);
            t->zc = yc[2];
            t->uc = yc[0] / yc[2];
            t->vc = yc[1] / yc[2];
            if (!(yc[2] > 0)) {  /* behind the camera: not drawn */
                t->ix0 = 0; t->ix1 = -1; t->iy0 = 0; t->iy1 = -1;
                return 1;
            }
            /* the pixels whose ray meets the support disc: the window box of
             * the disc's bounding square (all of it in front of the camera
             * when 2h < z_c), widened by a pixel; else the whole window */
            const double R2 = 2.0 * t->hh;
            double du = P->extent[0] / P->width, dv = P->extent[1] / P->height;
            double ul = -0.5 * P->extent[0], vb = -0.5 * P->extent[1];
            if (R2 >= yc[2]) {
                t->ix0 = 0; t->ix1 = P->width - 1; t->iy0 = 0; t->iy1 = P->height - 1;
                return 1;
            }
            /* on the billboard's plane the disc spans (x_c +- 2h, y_c +- 2h) */
            double umin = (yc[0] - R2) / yc[2], umax = (yc[0] + R2) / yc[2];
            double vmin = (yc[1] - R2) / yc[2], vmax = (yc[1] + R2) / yc[2];
            t->ix0 = (int64_t)ceil((umin - ul) / du - 0.5) - 1;
            t->ix1 = (int64_t)floor((umax - ul) / du - 0.5) + 1;
            t->iy0 = (int64_t)ceil((vmin - vb) / dv - 0.5) - 1;
            t->iy1 = (int64_t)floor((vmax - vb) / dv - 0.5) + 1;
            if (t->ix0 < 0) t->ix0 = 0;
            if (t->iy0 < 0) t->iy0 = 0;
            if (t->ix1 > P->width - 1) t->ix1 = P->width - 1;
            if (t->iy1 > P->height - 1) t->iy1 = P->height - 1;
            return 1;
        }
    }
    double pu[4], pv[4];  /* the vertices on the image plane */
    int behind = 0;
    for (int m = 0; m < 4; ++m) {
        if (P->perspective) {
            if (!(yv[m][2] > 0)) behind = 1;
            pu[m] = yv[m][0] / yv[m][2];
            pv[m] = yv[m][1] / yv[m][2];
        } else {
            pu[m] = yv[m][0];
            pv[m] = yv[m][1];
        }
    }
    if (behind) {  /* a vertex at or behind the camera plane: any pixel may see it */
        t->ix0 = 0; t->ix1 = P->width - 1;
        t->iy0 = 0; t->iy1 = P->height - 1;
        return 1;
    }
    double umin = pu[0], umax = pu[0], vmin = pv[0], vmax = pv[0];
    for (int m = 1; m < 4; ++m) {
        if (pu[m] < umin) umin = pu[m];
        if (pu[m] > umax) umax = pu[m];
        if (pv[m] < vmin) vmin = pv[m];
        if (pv[m] > vmax) vmax = pv[m];
    }
    double du = P->extent[0] / P->width, dv = P->extent[1] / P->height;
    double ul = -0.5 * P->extent[0], vb = -0.5 * P->extent[1];
    /* pixel centres inside [umin, umax], widened by one pixel on each side;
     * the clip itself decides the boundary pixels */
    t->ix0 = (int64_t)ceil((umin - ul) / du - 0.5) - 1;
    t->ix1 = (int64_t)floor((umax - ul) / du - 0.5) + 1;
    t->iy0 = (int64_t)ceil((vmin - vb) / dv - 0.5) - 1;
    t->iy1 = (int64_t)floor((vmax - vb) / dv - 0.5) + 1;
    return 1;
}

static double splat_w(double r, double h);

/* Length of the camera ray through (pu, pv) inside the tetrahedron. */
static double clip_dl_persp(const orc_tet *t, double pu, double pv) {
    if (t->splat) {  /* a billboard: the kernel where the ray crosses its plane */
        const double du = pu - t->uc, dv = pv - t->vc;
        return splat_w(t->zc * sqrt(du * du + dv * dv), t->hh);
    }
    double lo = 0.0, hi = INFINITY;  /* the half-line s >= 0 */
    for (int f = 0; f < 4; ++f) {
        double nd = t->n[f][0] * pu + t->n[f][1] * pv + t->n[f][2];
        if (nd > 0) {
            double q = t->h[f] / nd;
            if (q < hi) hi = q;
        } else if (nd < 0) {
            double q = t->h[f] / nd;
            if (q > lo) lo = q;
        } else {
            if (t->h[f] < 0) return 0.0;
            if (t->h[f] == 0 && !(t->n[f][0] < 0 || (t->n[f][0] == 0 && t->n[f][1] < 0))) return 0.0;
        }
    }
    if (!(hi > lo) || isinf(hi)) return 0.0;
    return (hi - lo) * sqrt(pu * pu + pv * pv + 1.0);
}

/* Length of the ray at pixel centre (pu, pv) inside the tetrahedron. */
static double clip_dl(const orc_tet *t, double pu, double pv) {
    if (t->persp) return clip_dl_persp(t, pu, pv);
    double lo = -INFINITY, hi = INFINITY;
    for (int f = 0; f < 4; ++f) {
        double nd = t->n[f][2];
        double s = t->h[f] - t->n[f][0] * pu - t->n[f][1] * pv;
        if (nd > 0) {
            double q = s / nd;
            if (q < hi) hi = q;
        } else if (nd < 0) {
            double q = s / nd;
            if (q > lo) lo = q;
        } else {
            if (s < 0) return 0.0;
            if (s == 0 && !(t->n[f][0] < 0 || (t->n[f][0] == 0 && t->n[f][1] < 0))) return 0.0;
        }
    }
    if (!(hi > lo) || isinf(lo) || isinf(hi)) return 0.0;
    /* slab: the part of the chord at depths in [s0, s1] */
    if (lo < t->s0) lo = t->s0;
    if (hi > t->s1) hi = t->s1;
    return hi > lo ? hi - lo : 0.0;
}

static inline double pixel_u(const orc_problem *P, int64_t ix) {
    return -0.5 * P->extent[0] + ((double)ix + 0.5) * (P->extent[0] / P->width);
}
static inline double pixel_v(const orc_problem *P, int64_t iy) {
    return -0.5 * P->extent[1] + ((double)iy + 0.5) * (P->extent[1] / P->height);
}

/* Map an unwrapped pixel index to the image; -1 when it falls outside. */
static inline int64_t map_col(const orc_problem *P, int64_t ix) {
    if (P->wrap) return imod(ix, P->width);
    return (ix >= 0 && ix < P->width) ? ix : -1;
}
static inline int64_t map_row(const orc_problem *P, int64_t iy) {
    if (P->wrap) return imod(iy, P->height);
    return (iy >= 0 && iy < P->height) ? iy : -1;
}

/* ------------------------------------------------------------ public API */

int orc_version(void) { return 1; }

/* Volumes of the six tetrahedra of one cube and their unwrapped vertices
 * (world coordinates), for connectivity checks.  verts: 6*4*3 doubles. */
int orc_cube_tets(const orc_problem *P, const float *x, const float *y, const float *z,
                  int64_t cube, double *verts, double *vols) {
    if (check_problem(P) != ORC_OK || !x || !y || !z) return ORC_EINVAL;
    if (cube < 0 || cube >= n_cubes(P)) return ORC_EINVAL;
    double X[8][3];
    cube_corners(P, x, y, z, cube, X);
    for (int t = 0; t < 6; ++t) {
        double v[4][3];
        for (int m = 0; m < 4; ++m)
            for (int q = 0; q < 3; ++q) {
                v[m][q] = X[TET_TABLE[t][m]][q];
                if (verts) verts[(t * 4 + m) * 3 + q] = v[m][q];
            }
        if (vols) vols[t] = signed_volume(v);
    }
    return ORC_OK;
}

/* Per-tet projection of an explicit list of tetrahedra (world vertices,
 * tet-major [T][4][3]) with per-tet masses; the lattice fields of P are
 * ignored.  out: H*W doubles, overwritten.  Serial, in list order. */
/* ---------------------------------------------------- centroid splatting
 * The centroid section's renderer: every tetrahedron T is drawn as a 2D
 * cubic-spline kernel centred on its centroid c_T (the mean of its four
 * vertices), of size h_T proportional to (m / rho_T)^(1/3) = |V(T)|^(1/3)
 * (proportionality constant 1), carrying q(T) |V(T)| (its mass for q = rho):
 *
 *   I(p) += q |V| W(|p - c_T|, h),
 *   W(r, h) = 10 / (7 pi h^2) * { 1 - 3/2 s^2 + 3/4 s^3   (0 <= s < 1)
 *                               { 1/4 (2 - s)^3          (1 <= s < 2)
 *                               { 0                       (s >= 2),  s = r / h,
 *
 * the 2D cubic spline normalised to a unit integral over the plane; p and c
 * in view-plane world coordinates, point-sampled at pixel centres (with the
 * pixel index modulo (W, H) under wrap).  fragments counts (pixel, T) with
 * W > 0.  Plain loops over tetrahedra in id order, one thread. */
static const double ORC_PI = 3.14159265358979323846;

static double splat_w(double r, double h) {
    const double s = r / h;
    const double c = 10.0 / (7.0 * ORC_PI * h * h);
    if (s < 1.0) return c * (1.0 - 1.5 * s * s + 0.75 * s * s * s);
    if (s < 2.0) return c * 0.25 * (2.0 - s) * (2.0 - s) * (2.0 - s);
    return 0.0;
}

static void splat_one(const orc_problem *P, const double v[4][3], double mass, double *out,
                      double *comp, orc_stats *s) {
    const double V = signed_volume(v);
    if (V == 0.0) { s->zero_volume++; return; }
    s->tets++;
    if (V > 0) s->inverted++;
    const double vol = fabs(V);
    const double rho = mass / vol;
    const double q = P->qpow == 0 ? 1.0 : (P->qpow == 1 ? rho : rho * rho);
    const double h = cbrt(vol);
    double cw[3] = {0, 0, 0};
    for (int m = 0; m < 4; ++m)
        for (int a = 0; a < 3; ++a) cw[a] += 0.25 * v[m][a];
    const double d[3] = {cw[0] - P->center[0], cw[1] - P->center[1], cw[2] - P->center[2]};
    const double cu = P->rot[0] * d[0] + P->rot[1] * d[1] + P->rot[2] * d[2];
    const double cv = P->rot[3] * d[0] + P->rot[4] * d[1] + P->rot[5] * d[2];
    const double du = P->extent[0] / P->width, dv = P->extent[1] / P->height;
    const double ul = -0.5 * P->extent[0], vb = -0.5 * P->extent[1];
    const int64_t ix0 = (int64_t)ceil((cu - 2 * h - ul) / du - 0.5), ix1 = (int64_t)floor((cu + 2 * h - ul) / du - 0.5);
    const int64_t iy0 = (int64_t)ceil((cv - 2 * h - vb) / dv - 0.5), iy1 = (int64_t)floor((cv + 2 * h - vb) / dv - 0.5);
    for (int64_t iy = iy0; iy <= iy1; ++iy) {
        const int64_t ry = map_row(P, iy);
        if (ry < 0) continue;
        const double pv = pixel_v(P, iy);
        for (int64_t ix = ix0; ix <= ix1; ++ix) {
            const int64_t rx = map_col(P, ix);
            if (rx < 0) continue;
            const double pu = pixel_u(P, ix);
            const double w = splat_w(sqrt((pu - cu) * (pu - cu) + (pv - cv) * (pv - cv)), h);
            if (w > 0) {
                s->fragments++;
                neu_add(&out[ry * P->width + rx], &comp[ry * P->width + rx], q * vol * w);
            }
        }
    }
}

int orc_splat_image(const orc_problem *P, const float *x, const float *y, const float *z, double *out,
                    orc_stats *st) {
    if (check_problem(P) != ORC_OK || P->perspective || !x || !y || !z || !out) return ORC_EINVAL;
    const int64_t ncube = n_cubes(P);
    const double mass = P->total_mass / (double)(6 * ncube);
    const int64_t npx = (int64_t)P->width * P->height;
    double *comp = (double *)calloc((size_t)npx, sizeof(double));
    if (!comp) return ORC_ENOMEM;
    memset(out, 0, sizeof(double) * (size_t)npx);
    orc_stats s = {0, 0, 0, 0};
    for (int64_t c = 0; c < ncube; ++c) {
        double X[8][3];
        cube_corners(P, x, y, z, c, X);
        for (int t = 0; t < 6; ++t) {
            double v[4][3];
            for (int m = 0; m < 4; ++m)
                for (int a = 0; a < 3; ++a) v[m][a] = X[TET_TABLE[t][m]][a];
            splat_one(P, v, mass, out, comp, &s);
        }
    }
    for (int64_t p = 0; p < npx; ++p) out[p] += comp[p];
    free(comp);
    if (st) *st = s;
    return ORC_OK;
}

/* Splats of an explicit tetrahedron list (world vertices [T][4][3], masses). */
int orc_splat_tets(const orc_problem *P, int64_t ntet, const double *verts, const double *mass,
                   double *out, orc_stats *st) {
    if (!P || P->width < 1 || P->height < 1 || !(P->extent[0] > 0) || !(P->extent[1] > 0) ||
        P->qpow < 0 || P->qpow > 2 || P->perspective || ntet < 0 || (ntet > 0 && (!verts || !mass)) || !out)
        return ORC_EINVAL;
    const int64_t npx = (int64_t)P->width * P->height;
    double *comp = (double *)calloc((size_t)npx, sizeof(double));
    if (!comp) return ORC_ENOMEM;
    memset(out, 0, sizeof(double) * (size_t)npx);
    orc_stats s = {0, 0, 0, 0};
    for (int64_t t = 0; t < ntet; ++t) {
        double v[4][3];
        memcpy(v, verts + t * 12, sizeof(v));
        splat_one(P, v, mass[t], out, comp, &s);
    }
    for (int64_t p = 0; p < npx; ++p) out[p] += comp[p];
    free(comp);
    if (st) *st = s;
    return ORC_OK;
}

int orc_project_tets(const orc_problem *P, int64_t ntet, const double *verts,
                     const double *mass, double *out, orc_stats *st) {
    if (!P || P->width < 1 || P->height < 1 || !(P->extent[0] > 0) || !(P->extent[1] > 0) ||
        P->qpow < 0 || P->qpow > 2 || (P->perspective && (P->wrap || P->slab)) || P->method < 0 ||
        P->method > 2 || (P->method && !P->perspective) ||
        (P->method == 2 && !(P->lod_radius >= 0.0 && isfinite(P->lod_radius))))
        return ORC_EINVAL;
    if (ntet < 0 || (ntet > 0 && (!verts || !mass)) || !out) return ORC_EINVAL;
    int64_t npx = (int64_t)P->width * P->height;
    double *comp = (double *)calloc((size_t)npx, sizeof(double));
    if (!comp) return ORC_ENOMEM;
    memset(out, 0, sizeof(double) * (size_t)npx);
    orc_stats s = {0, 0, 0, 0};
    for (int64_t t = 0; t < ntet; ++t) {
        double v[4][3];
        memcpy(v, verts + t * 12, sizeof(v));
        orc_tet tt;
        double V;
        if (!tet_setup(P, v, mass[t], &tt, &V)) { s.zero_volume++; continue; }
        s.tets++;
        if (V > 0) s.inverted++;
        for (int64_t iy = tt.iy0; iy <= tt.iy1; ++iy) {
            int64_t ry = map_row(P, iy);
            if (ry < 0) continue;
            double pv = pixel_v(P, iy);
            for (int64_t ix = tt.ix0; ix <= tt.ix1; ++ix) {
                int64_t rx = map_col(P, ix);
                if (rx < 0) continue;
                double dl = clip_dl(&tt, pixel_u(P, ix), pv);
                if (dl > 0) {
                    s.fragments++;
                    neu_add(&out[ry * P->width + rx], &comp[ry * P->width + rx], tt.q * dl);
                }
            }
        }
    }
    for (int64_t p = 0; p < npx; ++p) out[p] += comp[p];
    free(comp);
    if (st) *st = s;
    return ORC_OK;
}

/* Region mode: the image rectangle [cx0, cx0+cw) x [cy0, cy0+ch) of the
 * full projection.  out: ch*cw doubles, row-major, overwritten. */
/* The unwrapped indices i in [lo, hi] whose image index (i modulo n under
 * wrap, i itself otherwise) lies in the window [c0, c0 + cw): they form the
 * runs [c0 + k n, c0 + cw - 1 + k n] for k = *k0 .. *k1 (k = 0 only without
 * wrap), each clipped to [lo, hi]. */
static void window_periods(int wrap, int64_t lo, int64_t hi, int64_t c0, int64_t cw, int64_t n,
                           int64_t *k0, int64_t *k1) {
    if (!wrap) { *k0 = 0; *k1 = (lo <= c0 + cw - 1 && hi >= c0) ? 0 : -1; return; }
    int64_t a = lo - (c0 + cw - 1), b = hi - c0;  /* k n in [a, b] */
    *k0 = a >= 0 ? (a + n - 1) / n : -((-a) / n);
    *k1 = b >= 0 ? b / n : -((-b + n - 1) / n);
}

/* Region mode: the crop [cx0, cx0 + cw) x [cy0, cy0 + ch) of the image.
 * Every pixel sums the tetrahedra covering it in tetrahedron-id order, so the
 * result does not depend on the crop, the band height or the thread count;
 * tetrahedra and pixels outside the crop are only skipped. */
int orc_project_region(const orc_problem *P, const float *x, const float *y, const float *z,
                       int32_t cx0, int32_t cy0, int32_t cw, int32_t ch, double *out,
                       orc_stats *st, int32_t nthreads) {
    if (check_problem(P) != ORC_OK || !x || !y || !z || !out) return ORC_EINVAL;
    if (cx0 < 0 || cy0 < 0 || cw < 1 || ch < 1 || cx0 + cw > P->width || cy0 + ch > P->height)
        return ORC_EINVAL;
    if (nthreads < 1) nthreads = omp_get_max_threads();
    const int64_t ncube = n_cubes(P);
    const int64_t ntet = 6 * ncube;
    const double mass = P->total_mass / (double)ntet;
    /* rows per band: about 64 bands, at least 4 rows each (the listing below
     * holds one entry per tetrahedron and band) */
    const int BH = ch / 64 > 4 ? ch / 64 : 4;
    const int64_t nband = (ch + BH - 1) / BH;

    /* pass 1: candidate pixel range of every tetrahedron, and the counts */
    int32_t *r0 = (int32_t *)malloc(sizeof(int32_t) * (size_t)ntet);
    int32_t *r1 = (int32_t *)malloc(sizeof(int32_t) * (size_t)ntet);
    int32_t *q0 = (int32_t *)malloc(sizeof(int32_t) * (size_t)ntet);
    int32_t *q1 = (int32_t *)malloc(sizeof(int32_t) * (size_t)ntet);
    if (!r0 || !r1 || !q0 || !q1) { free(r0); free(r1); free(q0); free(q1); return ORC_ENOMEM; }
    int64_t zero_v = 0, inv = 0, live = 0;
#pragma omp parallel for schedule(static) num_threads(nthreads) reduction(+ : zero_v, inv, live)
    for (int64_t c = 0; c < ncube; ++c) {
        double X[8][3];
        cube_corners(P, x, y, z, c, X);
        for (int t = 0; t < 6; ++t) {
            double v[4][3];
            for (int m = 0; m < 4; ++m)
                for (int q = 0; q < 3; ++q) v[m][q] = X[TET_TABLE[t][m]][q];
            orc_tet tt;
            double V;
            int64_t id = 6 * c + t;
            r0[id] = 1; r1[id] = 0;
            if (!tet_setup(P, v, mass, &tt, &V)) {
                zero_v++;
                continue;
            }
            live++;
            if (V > 0) inv++;
            int64_t k0, k1;
            window_periods(P->wrap, tt.ix0, tt.ix1, cx0, cw, P->width, &k0, &k1);
            if (k0 > k1) continue;  /* no column in the crop */
            r0[id] = (int32_t)tt.iy0;
            r1[id] = (int32_t)tt.iy1;
            q0[id] = (int32_t)tt.ix0;
            q1[id] = (int32_t)tt.ix1;
        }
    }

    /* band lists in tet-id order (each tet at most once per band) */
    int64_t *cnt = (int64_t *)calloc((size_t)nband + 1, sizeof(int64_t));
    int64_t *stamp = (int64_t *)malloc(sizeof(int64_t) * (size_t)nband);
    if (!cnt || !stamp) {
        free(r0); free(r1); free(q0); free(q1); free(cnt); free(stamp);
        return ORC_ENOMEM;
    }
    for (int64_t b = 0; b < nband; ++b) stamp[b] = -1;
#define FOR_TET_BANDS(BODY)                                                   \
    for (int64_t id = 0; id < ntet; ++id) {                                   \
        if (r0[id] > r1[id]) continue;                                        \
        int64_t k0, k1;                                                       \
        window_periods(P->wrap, r0[id], r1[id], cy0, ch, P->height, &k0, &k1); \
        for (int64_t k = k0; k <= k1; ++k) {                                  \
            int64_t lo = cy0 + k * P->height, hi = lo + ch - 1;               \
            if (lo < r0[id]) lo = r0[id];                                     \
            if (hi > r1[id]) hi = r1[id];                                     \
            for (int64_t iy = lo; iy <= hi; ++iy) {                           \
                int64_t b = (iy - k * P->height - cy0) / BH;                  \
                if (stamp[b] == id) continue;                                 \
                stamp[b] = id;                                                \
                BODY                                                          \
            }                                                                 \
        }                                                                     \
    }
    FOR_TET_BANDS(cnt[b + 1]++;)
    for (int64_t b = 0; b < nband; ++b) cnt[b + 1] += cnt[b];
    int64_t npair = cnt[nband];
    int64_t *lst = (int64_t *)malloc(sizeof(int64_t) * (size_t)(npair > 0 ? npair : 1));
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)nband);
    if (!lst || !fill) {
        free(r0); free(r1); free(q0); free(q1); free(cnt); free(stamp); free(lst); free(fill);
        return ORC_ENOMEM;
    }
    for (int64_t b = 0; b < nband; ++b) { fill[b] = cnt[b]; stamp[b] = -1; }
    FOR_TET_BANDS(lst[fill[b]++] = id;)
#undef FOR_TET_BANDS
    free(fill);
    free(stamp);
    free(q0);
    free(q1);

    /* pass 2: every band, tetrahedra in id order, the crop's pixels only */
    double *comp = (double *)calloc((size_t)cw * ch, sizeof(double));
    if (!comp) { free(r0); free(r1); free(cnt); free(lst); return ORC_ENOMEM; }
    memset(out, 0, sizeof(double) * (size_t)cw * ch);
    int64_t frags = 0;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads) reduction(+ : frags)
    for (int64_t b = 0; b < nband; ++b) {
        int64_t row_lo = cy0 + b * BH, row_hi = cy0 + (b + 1) * BH;
        if (row_hi > cy0 + ch) row_hi = cy0 + ch;
        int64_t last_cube = -1;
        double X[8][3];
        for (int64_t e = cnt[b]; e < cnt[b + 1]; ++e) {
            int64_t id = lst[e];
            int64_t c = id / 6;
            int t = (int)(id % 6);
            if (c != last_cube) { cube_corners(P, x, y, z, c, X); last_cube = c; }
            double v[4][3];
            for (int m = 0; m < 4; ++m)
                for (int q = 0; q < 3; ++q) v[m][q] = X[TET_TABLE[t][m]][q];
            orc_tet tt;
            double V;
            if (!tet_setup(P, v, mass, &tt, &V)) continue;
            int64_t ky0, ky1, kx0, kx1;
            window_periods(P->wrap, tt.iy0, tt.iy1, row_lo, row_hi - row_lo, P->height, &ky0, &ky1);
            window_periods(P->wrap, tt.ix0, tt.ix1, cx0, cw, P->width, &kx0, &kx1);
            for (int64_t ky = ky0; ky <= ky1; ++ky) {
                int64_t ylo = row_lo + ky * P->height, yhi = row_hi - 1 + ky * P->height;
                if (ylo < tt.iy0) ylo = tt.iy0;
                if (yhi > tt.iy1) yhi = tt.iy1;
                for (int64_t iy = ylo; iy <= yhi; ++iy) {
                    int64_t ry = iy - ky * P->height;
                    double pv = pixel_v(P, iy);
                    for (int64_t kx = kx0; kx <= kx1; ++kx) {
                        int64_t xlo = cx0 + kx * P->width, xhi = cx0 + cw - 1 + kx * P->width;
                        if (xlo < tt.ix0) xlo = tt.ix0;
                        if (xhi > tt.ix1) xhi = tt.ix1;
                        for (int64_t ix = xlo; ix <= xhi; ++ix) {
                            int64_t rx = ix - kx * P->width;
                            double dl = clip_dl(&tt, pixel_u(P, ix), pv);
                            if (dl > 0) {
                                frags++;
                                int64_t o = (ry - cy0) * cw + (rx - cx0);
                                neu_add(&out[o], &comp[o], tt.q * dl);
                            }
                        }
                    }
                }
            }
        }
    }
    for (int64_t p = 0; p < (int64_t)cw * ch; ++p) out[p] += comp[p];
    free(comp);
    free(r0); free(r1); free(cnt); free(lst);
    if (st) {
        st->tets = live;
        st->zero_volume = zero_v;
        st->inverted = inv;
        st->fragments = frags;
    }
    return ORC_OK;
}

/* Pixel-sample mode: the projection at n listed pixels (px[s], py[s]),
 * each 0 <= px < W, 0 <= py < H.  out: n doubles. */
typedef struct { int32_t row, col, idx; } orc_sample;

static int cmp_sample(const void *a, const void *b) {
    const orc_sample *p = (const orc_sample *)a, *q = (const orc_sample *)b;
    if (p->row != q->row) return p->row < q->row ? -1 : 1;
    if (p->col != q->col) return p->col < q->col ? -1 : 1;
    return p->idx < q->idx ? -1 : (p->idx > q->idx);
}

int orc_project_pixels(const orc_problem *P, const float *x, const float *y, const float *z,
                       int64_t n, const int32_t *px, const int32_t *py, double *out,
                       orc_stats *st, int32_t nthreads) {
    if (check_problem(P) != ORC_OK || !x || !y || !z || !out || n < 0) return ORC_EINVAL;
    if (n > 0 && (!px || !py)) return ORC_EINVAL;
    for (int64_t s = 0; s < n; ++s)
        if (px[s] < 0 || px[s] >= P->width || py[s] < 0 || py[s] >= P->height) return ORC_EINVAL;
    if (nthreads < 1) nthreads = omp_get_max_threads();
    orc_sample *smp = (orc_sample *)malloc(sizeof(orc_sample) * (size_t)(n > 0 ? n : 1));
    if (!smp) return ORC_ENOMEM;
    for (int64_t s = 0; s < n; ++s) { smp[s].row = py[s]; smp[s].col = px[s]; smp[s].idx = (int32_t)s; }
    qsort(smp, (size_t)n, sizeof(orc_sample), cmp_sample);
    /* first sample index of every image row */
    int64_t *rowstart = (int64_t *)malloc(sizeof(int64_t) * ((size_t)P->height + 1));
    double *acc = (double *)calloc((size_t)nthreads * (size_t)(n > 0 ? n : 1) * 2, sizeof(double));
    if (!rowstart || !acc) { free(smp); free(rowstart); free(acc); return ORC_ENOMEM; }
    {
        int64_t s = 0;
        for (int64_t r = 0; r <= P->height; ++r) {
            while (s < n && smp[s].row < r) ++s;
            rowstart[r] = s;
        }
    }
    const int64_t ncube = n_cubes(P);
    const double mass = P->total_mass / (double)(6 * ncube);
    int64_t zero_v = 0, inv = 0, live = 0, frags = 0;
#pragma omp parallel num_threads(nthreads) reduction(+ : zero_v, inv, live, frags)
    {
        int tid = omp_get_thread_num();
        double *a = acc + (size_t)tid * (size_t)(n > 0 ? n : 1) * 2;
#pragma omp for schedule(static)
        for (int64_t c = 0; c < ncube; ++c) {
            double X[8][3];
            cube_corners(P, x, y, z, c, X);
            for (int t = 0; t < 6; ++t) {
                double v[4][3];
                for (int m = 0; m < 4; ++m)
                    for (int q = 0; q < 3; ++q) v[m][q] = X[TET_TABLE[t][m]][q];
                orc_tet tt;
                double V;
                if (!tet_setup(P, v, mass, &tt, &V)) { zero_v++; continue; }
                live++;
                if (V > 0) inv++;
                for (int64_t iy = tt.iy0; iy <= tt.iy1; ++iy) {
                    int64_t ry = map_row(P, iy);
                    if (ry < 0) continue;
                    if (rowstart[ry] == rowstart[ry + 1]) continue;
                    double pv = pixel_v(P, iy);
                    for (int64_t s = rowstart[ry]; s < rowstart[ry + 1]; ++s) {
                        int64_t col = smp[s].col;
                        /* every unwrapped column of the tet that lands on col */
                        int64_t first = P->wrap ? tt.ix0 + imod(col - tt.ix0, P->width) : col;
                        int64_t stride = P->wrap ? P->width : (int64_t)1 << 40;
                        for (int64_t ix = first; ix <= tt.ix1; ix += stride) {
                            if (ix < tt.ix0) continue;
                            double dl = clip_dl(&tt, pixel_u(P, ix), pv);
                            if (dl > 0) {
                                frags++;
                                neu_add(&a[2 * smp[s].idx], &a[2 * smp[s].idx + 1], tt.q * dl);
                            }
                        }
                    }
                }
            }
        }
    }
    for (int64_t s = 0; s < n; ++s) {
        double sum = 0, cmp = 0;
        for (int th = 0; th < nthreads; ++th) {
            const double *a = acc + (size_t)th * (size_t)(n > 0 ? n : 1) * 2;
            neu_add(&sum, &cmp, a[2 * s]);
            neu_add(&sum, &cmp, a[2 * s + 1]);
        }
        out[s] = sum + cmp;
    }
    free(smp); free(rowstart); free(acc);
    if (st) {
        st->tets = live;
        st->zero_volume = zero_v;
        st->inverted = inv;
        st->fragments = frags;
    }
    return ORC_OK;
}
