// Host-compiled run of the projector's per-tetrahedron code (tess_tet.h): the
// same setup_cube / tet_tiles / raster_record functions the HIP kernels call,
// driven by plain loops on the CPU in the kernels' order of work (tile lists,
// work items of at most `chunk` entries, one tile accumulator per item added
// into the image-sized second-difference array, then the row sums).  Used by
// the CPU test suite to check the kernel arithmetic against the oracle without
// a GPU.  Test code only.
#include "tess_tet.h"

#include <cmath>
#include <cstring>
#include <vector>

using namespace tess;

// The edge raster's split drawing: the first tile copy's kinks from the
// edge job (rows r0 .. r0 + cnt - 1, the terms the kernel's 16-lane groups
// compute) and that copy's seam line, then the pair routine for the further
// copies.
template <typename Dep, typename Seam, typename SeamRange>
static uint32_t split_pair(const EdgePayload &E, uint32_t eid, const BinParams &B, int tx0, int ty0, int n, int rows,
                           Dep &&dep, Seam &&seam, SeamRange &&seam_range, uint32_t &kinks) {
    const EdgeJob J = edge_job(E, B, tx0, ty0, n, rows, kinks);
    const int klo = J.shift - 3, khi = J.shift + n - 1;
    for (int s = 0; s < J.cnt; ++s) {
        const double u = fma((double)(J.r0 + s), J.sl, J.base);
        const double fl = floor(u);
        const int k = std::min(std::max((int)fl, klo), khi) - J.shift;
        const double v1 = fma(J.D, fl - u, J.D);
        dep(J.ta + s, k + 1, v1, J.D - v1);
    }
    if (J.seamed)
        edge_copy_seam(E, eid, B, tx0, n, J.kx, J.shift, J.ta - J.r0, J.r0, J.r0 + J.cnt - 1,
                       E.sl != 0.0 ? fast_rcp(E.sl) : 0.0, seam, seam_range);
    if (J.more) return edge_pair<false, true>(E, eid, 0u, B, tx0, ty0, n, rows, dep, seam, seam_range, kinks);
    return 0u;
}

extern "C" int hc_pipeline(const float *x, const float *y, const float *z, const int32_t dims[3],
                           int32_t periodic, double total_mass, int32_t precision, const double rot[9],
                           const double center[3], const double extent[2], int32_t W, int32_t H,
                           int32_t wrap, int32_t tile_rows, int32_t tile_cols, int32_t chunk,
                           double crease_div, int32_t qpow, const double *slab, int32_t splat, int32_t persp, int32_t hybrid, double lod_radius,
                           int32_t edges, double *out64, float *out32,
                           long long *stats /* [tets, zero, inverted, fp64_dets, fragments, spans,
                                               pairs, items, crease_records, edged] */) {
    LatticeParams L;
    std::memset(&L, 0, sizeof(L));
    L.x = x; L.y = y; L.z = z;
    for (int a = 0; a < 3; ++a) {
        L.d[a] = dims[a];
        L.c[a] = periodic ? dims[a] : dims[a] - 1;
        L.box[a] = 1.0;
    }
    L.ncubes = (int64_t)L.c[0] * L.c[1] * L.c[2];
    L.periodic = periodic;
    L.tet_mass = total_mass / (6.0 * (double)L.ncubes);
    L.v0 = 1.0 / (6.0 * (double)L.ncubes);
    L.det_v0_frac = 1e-6;
    L.det_cond_k = (precision || qpow != 1 || slab || splat || persp) ? -1.0 : 1e3;
    ViewParams V;
    for (int i = 0; i < 9; ++i) V.rot[i] = rot[i];
    for (int i = 0; i < 3; ++i) V.center[i] = center[i];
    V.u_left = -0.5 * extent[0];
    V.v_bottom = -0.5 * extent[1];
    V.inv_du = W / extent[0];
    V.inv_dv = H / extent[1];
    V.inv_W = 1.0 / W;
    V.inv_H = 1.0 / H;
    V.mass_px = 6.0 * L.tet_mass * V.inv_du * V.inv_dv;
    V.crease_bmax = crease_div > 0 ? V.mass_px * (double)L.ncubes / ((double)W * H) / crease_div : -1.0;
    V.W = W; V.H = H; V.wrap = wrap; V.qpow = qpow;
    V.slab = slab ? 1 : 0;
    V.splat = splat;
    V.persp = persp;
    V.hybrid = hybrid;
    V.lod_radius = lod_radius;
    V.slab_t[0] = slab ? slab[0] : 0.0;
    V.slab_t[1] = slab ? slab[1] : 0.0;
    // q != rho: the crease threshold from the integral of q (as the library)
    double qsum = 0.0;
    V.qsum = nullptr;
    V.bmax_per_q = crease_div > 0 ? V.inv_du * V.inv_dv / ((double)W * H) / crease_div : -1.0;
    if (qpow == 2) V.crease_bmax *= L.tet_mass / L.v0;
    if (qpow == 0 && !slab && !splat && !persp) {
        for (int64_t cube = 0; cube < L.ncubes; ++cube) qsum += cube_qvol(L, V, cube);
        V.qsum = &qsum;
    }
    // the edge form (plain pyramids): seven edge records per lattice vertex after the tetrahedra
    V.edges = (edges && !persp && !splat && !slab) ? 1 : 0;
    const int64_t nvert = (int64_t)L.d[0] * L.d[1] * L.d[2];
    const int64_t ntet = 6 * L.ncubes + (V.edges ? 7 * nvert : 0);
    std::vector<RecHead> head(ntet);
    std::vector<Payload> coef(6 * L.ncubes);
    std::vector<EdgePayload> ecoef(V.edges ? 7 * nvert : 0);
    std::vector<double> kinks(V.edges ? 36 * nvert : 0);
    std::vector<uint8_t> sil(V.edges ? 36 * nvert : 0);
    V.kinks = V.edges ? kinks.data() : nullptr;
    V.sil = V.edges ? sil.data() : nullptr;
    V.own_cap = (uint64_t)(6 * L.ncubes);
    V.own = nullptr;
    V.spill = nullptr;
    long long tets = 0, zero = 0, inv = 0, dets = 0, creases = 0, edged = 0;
    for (int64_t cube = 0; cube < L.ncubes; ++cube) {
        CubeCounts cnt;
        // (records stay at 6 cube + t here, every one with a payload slot)
        auto emit = [&](int t, const RecHead &R, const Payload &P) {
            head[6 * cube + t] = R;
            if (R.flags & REC_VALID) coef[6 * cube + t] = P;
        };
        if (persp) setup_cube<kFormPersp>(L, V, cube, emit, cnt);
        else if (splat) setup_cube<kFormSplat>(L, V, cube, emit, cnt);
        else if (slab) setup_cube<kFormFace>(L, V, cube, emit, cnt);
        else if (V.edges && edges == 4) {
            // every tetrahedron by the general setup (the kernels' k_setup_rest path)
            uint32_t all = 0x3fu;
            setup_cube<kFormPyramid, true, 2>(L, V, cube, emit, cnt, &all);
        } else if (V.edges) setup_cube<kFormPyramid, true>(L, V, cube, emit, cnt);
        else setup_cube<kFormPyramid>(L, V, cube, emit, cnt);
        tets += cnt.n_tets; zero += cnt.n_zero; inv += cnt.n_inv; dets += cnt.n_dets;
        for (int t = 0; t < 6; ++t) {
            creases += (head[6 * cube + t].flags & (REC_CREASE | REC_EDGED)) ? 1 : 0;
            edged += (head[6 * cube + t].flags & REC_EDGED) ? 1 : 0;
        }
    }
    if (V.edges)
        for (int64_t v = 0; v < nvert; ++v)
            setup_vertex_edges(L, V, v, &head[6 * L.ncubes + v], &ecoef[v]);
    BinParams B;
    B.Th = tile_rows;
    B.Tw = tile_cols;
    B.ntx = (W + tile_cols - 1) / tile_cols;
    B.nty = (H + tile_rows - 1) / tile_rows;
    B.W = W; B.H = H; B.wrap = wrap;
    B.seg_len = (int32_t)ntet;
    B.nseg = 1;
    B.ntet = (uint32_t)ntet;
    B.slab_t[0] = V.slab_t[0];
    B.slab_t[1] = V.slab_t[1];
    B.direct = splat || persp;
    B.ext_u = extent[0];
    B.ext_v = extent[1];
    const int ntiles = B.ntx * B.nty;
    B.nkey = (splat || slab || persp || V.edges) ? 1 : 32;
    B.edges = V.edges;
    B.first_edge = (uint32_t)(6 * L.ncubes);
    B.seam = V.edges && wrap ? 1 : 0;
    B.groups = V.edges ? kinks.data() : nullptr;
    // per tile: its records in id order; every pair's work class in range
    std::vector<std::vector<uint32_t>> lists(ntiles);
    for (int64_t id = 0; id < ntet; ++id) {
        const RecHead &r = head[id];
        if (!(r.flags & REC_VALID)) continue;
        const TileRange tr = tet_tiles(r, B);
        for (int s = 0; s < tr.count; ++s) {
            const int tile = tet_tile(B, tr, s);
            const int cls = B.nkey > 1 ? pair_class(r, B, tile / B.ntx) : 0;
            if (cls < 0 || cls >= B.nkey || (cls != 0 && !(r.flags & REC_CREASE))) return -2;
            lists[tile].push_back((uint32_t)id);
        }
    }
    std::vector<double> acc((size_t)W * H, 0.0);
    std::vector<double> tile((size_t)tile_rows * tile_cols);
    std::vector<double> seam((size_t)2 * tile_rows);  // per tile row: the seam line a + b j
    long long frags = 0, spans = 0, pairs = 0, items = 0;
    for (int t = 0; t < ntiles; ++t) {
        const int tx0 = (t % B.ntx) * B.Tw, ty0 = (t / B.ntx) * B.Th;
        const int n = std::min(B.Tw, W - tx0), rows = std::min(B.Th, H - ty0);
        const std::vector<uint32_t> &lst = lists[t];
        pairs += (long long)lst.size();
        for (size_t first = 0; first < lst.size(); first += (size_t)chunk) {
            ++items;
            std::fill(tile.begin(), tile.end(), 0.0);
            std::fill(seam.begin(), seam.end(), 0.0);
            const size_t last = std::min(lst.size(), first + (size_t)chunk);
            for (size_t e = first; e < last; ++e) {
                const uint32_t id = lst[e];
                uint32_t sp = 0, kk = 0;
                const bool is_edge = V.edges && id >= B.first_edge;
                const double *cf = is_edge ? nullptr : coef[id].c;
                auto sl = [&](int row, double a, double b) {
                    if (row < 0 || row >= rows) throw 2;
                    seam[(size_t)row] += a;
                    seam[(size_t)tile_rows + row] += b;
                };
                auto rr = [&](auto &&dep) {
                    auto dep2 = [&](int row, int j, double a, double b) {
                        dep(row, j, a);
                        dep(row, j + 1, b);
                    };
                    auto slr = [&](int lo, int hi, double alpha, double beta, double gamma) {
                        if (lo < 0 || hi >= rows || lo > hi) throw 3;
                        for (int r = lo; r <= hi; ++r) sl(r, alpha + beta * (double)r, gamma);
                    };
                    return persp ? raster_record<kFormPersp>(head[id], cf, B, tx0, ty0, n, rows, dep, sl, sp, kk)
                         : splat ? raster_record<kFormSplat>(head[id], cf, B, tx0, ty0, n, rows, dep, sl, sp, kk)
                         : slab ? raster_record<kFormFace>(head[id], cf, B, tx0, ty0, n, rows, dep, sl, sp, kk)
                         : is_edge ? (edges == 3 ? split_pair(ecoef[id - B.first_edge], id - B.first_edge, B, tx0, ty0, n, rows,
                                                              dep2, sl, slr, kk)
                                      : edges == 2 ? edge_pair<false>(ecoef[id - B.first_edge], id - B.first_edge, 0u, B, tx0, ty0, n,
                                                                     rows, dep2, sl, slr, kk)
                                                 : edge_pair<true>(ecoef[id - B.first_edge], id - B.first_edge, head[id].spare, B, tx0, ty0, n,
                                                                   rows, dep2, sl, slr, kk))
                         : V.edges ? raster_record<kFormEdge>(head[id], cf, B, tx0, ty0, n, rows, dep, sl, sp, kk)
                                : raster_record<kFormPyramid>(head[id], cf, B, tx0, ty0, n, rows, dep, sl, sp, kk);
                };
                frags += (int32_t)rr(
                                     [&](int row, int j, double v) {
                                         if (row < 0 || row >= rows || j < -2 || j > n + 1) throw 1;
                                         if (j >= 0 && j < n) tile[(size_t)row * B.Tw + j] += v;
                                     });
                spans += sp;
            }
            for (int r = 0; r < rows; ++r) {
                for (int c = 0; c < n; ++c) acc[(size_t)(ty0 + r) * W + tx0 + c] += tile[(size_t)r * B.Tw + c];
                acc[(size_t)(ty0 + r) * W] += seam[(size_t)r];
                if (W > 1) acc[(size_t)(ty0 + r) * W + 1] += seam[(size_t)tile_rows + r] - seam[(size_t)r];
            }
        }
    }
    for (int iy = 0; iy < H; ++iy) {
        double d1 = 0.0, f = 0.0;
        for (int ix = 0; ix < W; ++ix) {
            d1 += acc[(size_t)iy * W + ix];
            f = (splat || persp) ? acc[(size_t)iy * W + ix] : f + d1;
            if (out64) out64[(size_t)iy * W + ix] = f;
            if (out32) out32[(size_t)iy * W + ix] = (float)std::fmax(f, 0.0);
        }
    }
    if (stats) {
        stats[0] = tets; stats[1] = zero; stats[2] = inv; stats[3] = dets;
        stats[4] = frags; stats[5] = spans; stats[6] = pairs; stats[7] = items; stats[8] = creases;
        stats[9] = edged;
    }
    return 0;
}

// floor_div_r against exact floor division over pixel-sized arguments, with
// its reciprocal moved `ulps` units in the last place either way (the GPU's
// reciprocal estimate is within one); returns the number of mismatches
extern "C" int64_t hc_floor_div_check(int ulps) {
    const int divisors[] = {1, 2, 3, 7, 16, 31, 32, 37, 64, 100, 128, 255, 256, 333, 512, 1000, 1024, 2048,
                            4096, 4097, 8191, 16384, 32767};
    int64_t bad = 0;
    for (int b : divisors)
        for (int sgn = -1; sgn <= 1; sgn += 2) {
            float rb = 1.0f / (float)b;
            for (int k = 0; k < ulps; ++k) rb = std::nextafter(rb, sgn > 0 ? 2.0f : 0.0f);
            for (int a = -70000; a <= 70000; ++a) {
                const int exact = a >= 0 ? a / b : -((-a + b - 1) / b);
                if (floor_div_r(a, b, rb) != exact) ++bad;
            }
        }
    return bad;
}
