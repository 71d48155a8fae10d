// Host-compiled run of the projector's per-tetrahedron code (tess_tet.h): the
// same setup_cube / tile_accept / eval_* functions the HIP kernels call,
// driven by plain loops on the CPU.  Used by the CPU test suite to check the
// kernel arithmetic against the oracle without a GPU.  Test code only.
#include "tess_tet.h"

#include <cstring>
#include <vector>

using namespace tess;

extern "C" int hc_project(const float *x, const float *y, const float *z, const int32_t dims[3],
                          int32_t periodic, double total_mass, const double rot[9],
                          const double center[3], const double extent[2], int32_t W, int32_t H,
                          int32_t wrap, double fp64_cond, int32_t tile, double *out,
                          long long *stats /* [tets, zero, inverted, fp64_tets, fragments,
                                               culled_but_covered] */) {
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
    L.det_cond_k = 1e3;
    L.fp64_cond = fp64_cond;
    ViewParams V;
    for (int i = 0; i < 9; ++i) V.rot[i] = rot[i];
    for (int i = 0; i < 3; ++i) V.center[i] = center[i];
    V.u_left = -0.5 * extent[0];
    V.v_bottom = -0.5 * extent[1];
    V.inv_du = W / extent[0];
    V.inv_dv = H / extent[1];
    V.mass_px = 6.0 * L.tet_mass * V.inv_du * V.inv_dv;
    V.W = W; V.H = H; V.wrap = wrap;
    BinParams B;
    B.T = tile;
    B.ntx = (W + tile - 1) / tile;
    B.nty = (H + tile - 1) / tile;
    B.W = W; B.H = H; B.wrap = wrap;
    std::vector<double> img((size_t)W * H, 0.0);
    long long tets = 0, zero = 0, inv = 0, f64 = 0, frags = 0, culled = 0;
    constexpr int LS = 16;  // strip length, as in the raster's 32- and 64-pixel tiles
    for (int64_t cube = 0; cube < L.ncubes; ++cube) {
        TetRec r[6];
        Footprint fp[6];
        bool want64[6];
        CubeCounts cnt;
        setup_cube(L, V, cube, r, fp, want64, cnt);
        tets += cnt.n_tets; zero += cnt.n_zero; inv += cnt.n_inv;
        for (int t = 0; t < 6; ++t) {
            if (!(r[t].h.flags & REC_VALID)) continue;
            f64 += want64[t] ? 1 : 0;
            const TetRec &R = r[t];
            // every image pixel of the footprint's box, evaluated in raster strips
            for (int gy = range_lo(R.h.by); gy <= range_hi(R.h.by); ++gy) {
                const int iy = wrap ? ((gy % H) + H) % H : gy;
                // strip starts aligned to LS in image coordinates, as lanes own them
                const int img_x0 = wrap ? ((range_lo(R.h.bx) % W) + W) % W : range_lo(R.h.bx);
                const int shift = range_lo(R.h.bx) - img_x0;  // record frame minus image frame
                for (int sx = (img_x0 / LS) * LS; sx + shift <= range_hi(R.h.bx); sx += LS) {
                    const int gx0 = sx + shift;
                    float accf[LS] = {0};
                    double accd[LS] = {0};
                    if (!want64[t]) {
                        const float xf = (float)(gx0 - range_lo(R.h.bx)) + 0.5f, yf = (float)(gy - range_lo(R.h.by)) + 0.5f;
                        eval_any<float, LS>(R.c, R.h.flags, xf, yf, accf);
                        frags += eval_general<float, LS, true>(R.c, R.h.flags, xf, yf, accf,
                                                               range_lo(R.h.bx) - gx0, range_hi(R.h.bx) - gx0);
                    } else {
                        const double xd = (double)(gx0 - range_lo(R.h.bx)) + 0.5, yd = (double)(gy - range_lo(R.h.by)) + 0.5;
                        eval_any<double, LS>(fp[t].c, R.h.flags, xd, yd, accd);
                        frags += eval_general<double, LS, true>(fp[t].c, R.h.flags, xd, yd, accd,
                                                                range_lo(R.h.bx) - gx0, range_hi(R.h.bx) - gx0);
                    }
                    for (int k = 0; k < LS; ++k) {
                        const int gx = gx0 + k;
                        const int ix = wrap ? ((gx % W) + W) % W : gx;
                        if (gx < range_lo(R.h.bx) || gx > range_hi(R.h.bx)) {
                            // outside the box (inside the image) the functions must vanish
                            const bool in_image = wrap || (gx >= 0 && gx < W);
                            if (in_image && (accf[k] != 0.f || accd[k] != 0.0)) return -100;
                            continue;
                        }
                        if (ix < 0 || ix >= W || iy < 0 || iy >= H) continue;
                        const double v = (double)accf[k] + accd[k];
                        img[(size_t)iy * W + ix] += v;
                        if (v > 0) {
                            TetRec Rt = R;
                            if (!want64[t]) Rt.h.flags &= ~REC_FP64; else Rt.h.flags |= REC_FP64;
                            if (!tile_accept(Rt, ix / B.T, iy / B.T, B)) ++culled;
                        }
                    }
                }
            }
        }
    }
    std::memcpy(out, img.data(), sizeof(double) * img.size());
    if (stats) {
        stats[0] = tets; stats[1] = zero; stats[2] = inv; stats[3] = f64; stats[4] = frags; stats[5] = culled;
    }
    return 0;
}

// The whole projection pipeline on the CPU with the kernels' own functions:
// setup_cube for every cube (FP64 slots handed out in id order), the stable
// per-tile lists of tet_tile, work items of at most `chunk` entries,
// raster_lane for every lane of every item, and the ordered finalize.
template <int T, int L>
static void raster_items(const std::vector<TetRec> &rec, const std::vector<Coef64> &coef,
                         const std::vector<uint32_t> &pairs, const std::vector<WorkItem> &items,
                         const BinParams &B, std::vector<double> &partials, long long &frags) {
    partials.assign(items.size() * T * T, 0.0);
    for (size_t i = 0; i < items.size(); ++i) {
        for (int tid = 0; tid < T * T / L; ++tid) {
            Acc<L> acc;
            unsigned f = 0, f4 = 0;
            raster_lane<T, L, true>(rec.data(), coef.data(), (uint32_t)coef.size(), pairs.data(), items[i], B,
                                    tid, acc, f, f4);
            frags += f;
            const int row = tid / (T / L), strip = tid % (T / L);
            for (int k = 0; k < L; ++k) partials[i * T * T + row * T + strip * L + k] = acc.d[k];
        }
    }
}

extern "C" int hc_pipeline(const float *x, const float *y, const float *z, const int32_t dims[3],
                           int32_t periodic, double total_mass, const double rot[9],
                           const double center[3], const double extent[2], int32_t W, int32_t H,
                           int32_t wrap, double fp64_cond, int32_t tile, int32_t chunk, float *out,
                           long long *stats /* [tets, fp64_tets, pairs, items, fragments] */) {
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
    L.det_cond_k = 1e3;
    L.fp64_cond = fp64_cond;
    ViewParams V;
    for (int i = 0; i < 9; ++i) V.rot[i] = rot[i];
    for (int i = 0; i < 3; ++i) V.center[i] = center[i];
    V.u_left = -0.5 * extent[0];
    V.v_bottom = -0.5 * extent[1];
    V.inv_du = W / extent[0];
    V.inv_dv = H / extent[1];
    V.mass_px = 6.0 * L.tet_mass * V.inv_du * V.inv_dv;
    V.W = W; V.H = H; V.wrap = wrap;
    const int64_t ntet = 6 * L.ncubes;
    std::vector<TetRec> rec(ntet);
    std::vector<Coef64> coef;
    long long tets = 0;
    for (int64_t cube = 0; cube < L.ncubes; ++cube) {
        TetRec r[6];
        Footprint fp[6];
        bool want64[6];
        CubeCounts cnt;
        setup_cube(L, V, cube, r, fp, want64, cnt);
        tets += cnt.n_tets;
        for (int t = 0; t < 6; ++t) {
            if (want64[t]) {
                r[t].h.flags |= REC_FP64;
                r[t].h.slot = (uint32_t)coef.size();
                Coef64 c;
                for (int g = 0; g < 12; ++g) c.c[g] = fp[t].c[g];
                coef.push_back(c);
            }
            rec[6 * cube + t] = r[t];
        }
    }
    BinParams B;
    B.T = tile;
    B.ntx = (W + tile - 1) / tile;
    B.nty = (H + tile - 1) / tile;
    B.W = W; B.H = H; B.wrap = wrap;
    B.seg_len = (int32_t)ntet;
    B.nseg = 1;
    B.ntet = (uint32_t)ntet;
    const int ntiles = B.ntx * B.nty;
    std::vector<std::vector<uint32_t>> lists(ntiles);
    for (int64_t id = 0; id < ntet; ++id) {
        const TetRec &r = rec[id];
        if (!(r.h.flags & REC_VALID)) continue;
        const TileRange tr = tet_tiles(r, B);
        for (int s = 0; s < tr.count; ++s) {
            int t;
            if (tet_tile(r, B, tr, s, t)) lists[t].push_back((uint32_t)id);
        }
    }
    std::vector<uint32_t> pairs;
    std::vector<WorkItem> items;
    std::vector<uint32_t> tile_items(ntiles + 1, 0);
    for (int t = 0; t < ntiles; ++t) {
        const uint64_t begin = pairs.size();
        pairs.insert(pairs.end(), lists[t].begin(), lists[t].end());
        tile_items[t] = (uint32_t)items.size();
        for (uint64_t f = begin; f < pairs.size(); f += (uint64_t)chunk) {
            WorkItem w;
            w.first = f;
            w.count = (uint32_t)std::min<uint64_t>((uint64_t)chunk, pairs.size() - f);
            w.tile = (uint32_t)t;
            items.push_back(w);
        }
    }
    tile_items[ntiles] = (uint32_t)items.size();
    std::vector<double> partials;
    long long frags = 0;
    if (tile == 16) raster_items<16, 4>(rec, coef, pairs, items, B, partials, frags);
    else if (tile == 32) raster_items<32, 16>(rec, coef, pairs, items, B, partials, frags);
    else if (tile == 64) raster_items<64, 16>(rec, coef, pairs, items, B, partials, frags);
    else return -1;
    for (int iy = 0; iy < H; ++iy)
        for (int ix = 0; ix < W; ++ix) {
            const int t = (iy / tile) * B.ntx + ix / tile;
            double s = 0.0;
            for (uint32_t it = tile_items[t]; it < tile_items[t + 1]; ++it)
                s += partials[(size_t)it * tile * tile + (iy % tile) * tile + ix % tile];
            out[(size_t)iy * W + ix] = (float)s;
        }
    if (stats) {
        stats[0] = tets; stats[1] = (long long)coef.size(); stats[2] = (long long)pairs.size();
        stats[3] = (long long)items.size(); stats[4] = frags;
    }
    return 0;
}
