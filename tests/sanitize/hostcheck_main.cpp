// Sanitizer driver of the host twin (test infrastructure): the kernels'
// per-tetrahedron code run by tests/hostcheck/hostcheck.cpp on small
// jittered lattices in every form, built with AddressSanitizer and
// UndefinedBehaviorSanitizer on the host side by tests/test_sanitizers.py.
// Exits 0 when every case succeeds with finite output.
#include "../hostcheck/hostcheck.cpp"

#include <cstdio>

int main() {
    const int N = 6;
    std::vector<float> x(N * N * N), y(N * N * N), z(N * N * N);
    uint64_t s = 88172645463325252ull;
    auto ur = [&]() {
        s = s * 6364136223846793005ull + 1442695040888963407ull;
        return (double)(s >> 11) / 9007199254740992.0;
    };
    for (int k = 0; k < N; ++k)
        for (int j = 0; j < N; ++j)
            for (int i = 0; i < N; ++i) {
                const int id = i + N * (j + N * k);
                x[id] = (float)std::fmod((i + 0.6 * (ur() - 0.5)) / N + 1.0, 1.0);
                y[id] = (float)std::fmod((j + 0.6 * (ur() - 0.5)) / N + 1.0, 1.0);
                z[id] = (float)std::fmod((k + 0.6 * (ur() - 0.5)) / N + 1.0, 1.0);
            }
    const int32_t dims[3] = {N, N, N};
    const double eye[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    const double rot[9] = {0.36, 0.48, -0.8, -0.8, 0.6, 0.0, 0.48, 0.64, 0.6};
    const double c[3] = {0.5, 0.5, 0.5}, cam[3] = {0.45, 0.52, -1.4};
    const double e1[2] = {1.0, 1.0}, e2[2] = {2.0, 2.0};
    const double slab[2] = {-0.2, 0.3};
    const int W = 50, H = 38;
    std::vector<double> out64((size_t)W * H);
    std::vector<float> out32((size_t)W * H);
    long long st[10];
    int fails = 0;
    struct Case {
        bool rotated;
        int qpow, tile_rows, tile_cols, edges, splat, persp, hybrid;
        const double *slab;
    };
    const Case cases[] = {
        {false, 1, 8, 16, 1, 0, 0, 0, nullptr}, {false, 1, 3, 37, 2, 0, 0, 0, nullptr},
        {false, 0, 8, 50, 0, 0, 0, 0, nullptr}, {true, 2, 4, 17, 1, 0, 0, 0, nullptr},
        {true, 1, 16, 16, 0, 0, 0, 0, nullptr}, {false, 1, 8, 16, 0, 0, 0, 0, slab},
        {false, 1, 8, 16, 0, 1, 0, 0, nullptr}, {true, 1, 8, 16, 0, 0, 1, 0, nullptr},
        {true, 1, 8, 16, 0, 1, 1, 0, nullptr},  {true, 1, 8, 16, 0, 0, 1, 1, nullptr},
    };
    for (const Case &k : cases) {
        const bool rotated = k.rotated || k.persp;
        const int rc = hc_pipeline(x.data(), y.data(), z.data(), dims, 1, 1.0, 0, rotated ? rot : eye,
                                   k.persp ? cam : c, rotated ? e2 : e1, W, H, rotated ? 0 : 1, k.tile_rows,
                                   k.tile_cols, 64, W / 64.0, k.qpow, k.slab, k.splat, k.persp, k.hybrid, 1.2,
                                   k.edges, out64.data(), out32.data(), st);
        bool finite = true;
        for (double v : out64) finite = finite && std::isfinite(v);
        fails += (rc != 0 || !finite) ? 1 : 0;
    }
    std::printf("host twin sanitizer driver: %d failures\n", fails);
    return fails != 0;
}
