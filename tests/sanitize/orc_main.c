/* Sanitizer driver of the FP64 oracle (test infrastructure): the oracle's
 * entry points on small jittered lattices, every view kind and a crop, built
 * with AddressSanitizer and UndefinedBehaviorSanitizer by
 * tests/test_sanitizers.py.  Exits 0 when every call succeeds with finite
 * output; the sanitizers abort on a memory or undefined-behaviour error. */
#include "../../oracle/tess_oracle.c"

#include <stdio.h>

static uint64_t lcg = 88172645463325252ull;
static double urand(void) {
    lcg = lcg * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(lcg >> 11) / 9007199254740992.0;
}

static int finite_all(const double *a, int64_t n) {
    for (int64_t i = 0; i < n; ++i)
        if (!isfinite(a[i])) return 0;
    return 1;
}

static void set_view(orc_problem *P, int rotated, int w, int h) {
    static const double eye[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    static const double rot[9] = {0.36, 0.48, -0.8, -0.8, 0.6, 0.0, 0.48, 0.64, 0.6};
    for (int i = 0; i < 9; ++i) P->rot[i] = rotated ? rot[i] : eye[i];
    for (int a = 0; a < 3; ++a) P->center[a] = 0.5;
    P->extent[0] = P->extent[1] = rotated ? 2.0 : 1.0;
    P->width = w;
    P->height = h;
    P->wrap = rotated ? 0 : 1;
}

int main(void) {
    enum { N = 6 };
    float x[N * N * N], y[N * N * N], z[N * N * N];
    for (int k = 0; k < N; ++k)
        for (int j = 0; j < N; ++j)
            for (int i = 0; i < N; ++i) {
                const int id = i + N * (j + N * k);
                x[id] = (float)fmod((i + 0.5 * (urand() - 0.5)) / N + 1.0, 1.0);
                y[id] = (float)fmod((j + 0.5 * (urand() - 0.5)) / N + 1.0, 1.0);
                z[id] = (float)fmod((k + 0.5 * (urand() - 0.5)) / N + 1.0, 1.0);
            }
    orc_problem P;
    memset(&P, 0, sizeof(P));
    P.dims[0] = P.dims[1] = P.dims[2] = N;
    P.box[0] = P.box[1] = P.box[2] = 1.0;
    P.periodic = 1;
    P.total_mass = 1.0;
    P.qpow = 1;
    double img[48 * 40], vals[7];
    orc_stats st;
    int fails = 0;
    for (int rotated = 0; rotated < 2; ++rotated)
        for (int qpow = 0; qpow < 3; ++qpow) {
            set_view(&P, rotated, 48, 40);
            P.qpow = qpow;
            fails += orc_project_region(&P, x, y, z, 0, 0, 48, 40, img, &st, 2) != 0 || !finite_all(img, 48 * 40);
            fails += orc_project_region(&P, x, y, z, 7, 5, 20, 17, img, &st, 3) != 0 || !finite_all(img, 20 * 17);
            const int32_t px[7] = {0, 47, 3, 20, 31, 47, 0}, py[7] = {0, 39, 5, 20, 11, 0, 39};
            fails += orc_project_pixels(&P, x, y, z, 7, px, py, vals, &st, 2) != 0 || !finite_all(vals, 7);
        }
    /* a depth slab, splats, a perspective camera with billboards and the hybrid */
    set_view(&P, 0, 48, 40);
    P.qpow = 1;
    P.slab = 1;
    P.slab_t[0] = -0.2;
    P.slab_t[1] = 0.3;
    fails += orc_project_region(&P, x, y, z, 0, 0, 48, 40, img, &st, 2) != 0 || !finite_all(img, 48 * 40);
    P.slab = 0;
    fails += orc_splat_image(&P, x, y, z, img, &st) != 0 || !finite_all(img, 48 * 40);
    set_view(&P, 1, 48, 40);
    P.wrap = 0;
    P.perspective = 1;
    P.center[0] = 0.45; P.center[1] = 0.52; P.center[2] = -1.4;
    for (int m = 0; m < 3; ++m) {
        P.method = m;
        P.lod_radius = 1.6;
        fails += orc_project_region(&P, x, y, z, 0, 0, 48, 40, img, &st, 2) != 0 || !finite_all(img, 48 * 40);
    }
    /* a non-periodic lattice */
    P.perspective = 0;
    P.method = 0;
    set_view(&P, 1, 48, 40);
    P.periodic = 0;
    fails += orc_project_region(&P, x, y, z, 0, 0, 48, 40, img, &st, 2) != 0 || !finite_all(img, 48 * 40);
    printf("oracle sanitizer driver: %d failures\n", fails);
    return fails != 0;
}
