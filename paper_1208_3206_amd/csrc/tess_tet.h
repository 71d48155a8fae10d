// Per-tetrahedron arithmetic of the projector, shared by the HIP kernels and
// by host-compiled checks of the same code (every function is host+device).
#pragma once

#include "tess_internal.h"

#include <cmath>
#include <cstdint>

#define TESS_HD __host__ __device__

namespace tess {

// ------------------------------------------------------------------ tables
// Connectivity of the six tetrahedra; cube corner n = a + 2b + 4c sits at
// lattice offset (a, b, c).
constexpr int kTet[6][4] = {{1, 0, 2, 4}, {3, 1, 2, 4}, {3, 5, 1, 4},
                                       {3, 6, 5, 4}, {3, 2, 6, 4}, {3, 7, 5, 6}};

// Face a of a tetrahedron is the one opposite vertex a; its vertices in
// increasing order.
constexpr int kFace[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};

// Edge (i, j), the other two vertices (k, l), and the signs s with
// cross(q_j - q_i, q_k - q_i) = sk * D[l] and cross(q_j - q_i, q_l - q_i) =
// sl * D[k], D[a] being the orientation of face a in kFace order.
struct EdgeInfo {
    int i, j, k, l, sk, sl;
};
constexpr EdgeInfo kEdge[6] = {{0, 1, 2, 3, +1, +1}, {0, 2, 1, 3, -1, +1},
                                          {0, 3, 1, 2, -1, -1}, {1, 2, 0, 3, +1, +1},
                                          {1, 3, 0, 2, +1, -1}, {2, 3, 0, 1, +1, +1}};


// ------------------------------------------------------------- utilities
TESS_HD inline int64_t imod64(int64_t a, int64_t m) {
    int64_t r = a % m;
    return r < 0 ? r + m : r;
}
TESS_HD inline int imod(int a, int m) {
    int r = a % m;
    return r < 0 ? r + m : r;
}
TESS_HD inline int floor_div(int a, int b) {  // b > 0
    return a >= 0 ? a / b : -((-a + b - 1) / b);
}
TESS_HD inline int ceil_div(int a, int b) {  // b > 0
    return -floor_div(-a, b);
}


// Volume determinant (times 6) in FP64, evaluated term by term without
// contraction so that an exact zero is decided the same way as by a plain
// left-to-right FP64 evaluation of Eq. Eqn:TetVolume.
TESS_HD __attribute__((noinline)) double det6_fp64(const double a[3], const double b[3], const double c[3]) {
#pragma clang fp contract(off)
    double cx = b[1] * c[2] - b[2] * c[1];
    double cy = b[2] * c[0] - b[0] * c[2];
    double cz = b[0] * c[1] - b[1] * c[0];
    return a[0] * cx + a[1] * cy + a[2] * cz;
}

// ------------------------------------------------------ footprint setup
struct Footprint {
    double c[12];
    int ng, nw;
    uint32_t ties;
    double cond;  // FP32 error amplification: max over the box of sum |terms| / peak
};

// Builds the G functions and walls of one tetrahedron from its projected
// vertices q (pixel units, relative to the record origin); X, Y are the
// record's box sizes in pixels.  Returns false when the projection has zero
// area (no pixel can receive anything).
TESS_HD inline bool footprint(const double qx[4], const double qy[4], double mass_px, double X,
                                 double Y, Footprint &fp) {
    double D[4];
    double sumD = 0.0;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const int b = kFace[a][0], c = kFace[a][1], d = kFace[a][2];
        const double ex = qx[c] - qx[b], ey = qy[c] - qy[b];
        const double fx = qx[d] - qx[b], fy = qy[d] - qy[b];
        D[a] = ex * fy - ey * fx;
        sumD += fabs(D[a]);
    }
    if (sumD == 0.0) return false;
    // the faces cover the silhouette twice, so its area is sum|D|/4 and the
    // apex value 3 m / area is 2 mass_px / sum|D|
    const double peak = 2.0 * mass_px / sumD;
    int ng = 0, nw = 0;
    uint32_t ties = 0;
    double cond = 0.0;
#pragma unroll
    for (int g = 0; g < 12; ++g) fp.c[g] = 0.0;
    // silhouette edges: q_k and q_l on the same side of edge (i, j)
#pragma unroll
    for (int e = 0; e < 6; ++e) {
        const EdgeInfo E = kEdge[e];
        const double ck = (double)E.sk * D[E.l];
        const double cl = (double)E.sl * D[E.k];
        if ((ck > 0 && cl > 0) || (ck < 0 && cl < 0)) {
            if (ng >= 4) return false;
            const double dx = qx[E.j] - qx[E.i], dy = qy[E.j] - qy[E.i];
            const double K = mass_px / (ck * fabs(cl));
            const double bb = -K * dy, cc = K * dx;
            const double aa = K * (dy * qx[E.i] - dx * qy[E.i]);
            fp.c[3 * ng + 0] = aa;
            fp.c[3 * ng + 1] = bb;
            fp.c[3 * ng + 2] = cc;
            cond = fmax(cond, (fabs(aa) + fabs(bb) * X + fabs(cc) * Y) / peak);
            ++ng;
        }
    }
    if (ng == 0) return false;
    // walls: faces seen edge-on (projected determinant exactly zero)
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        if (D[a] != 0.0) continue;
        const int f0 = kFace[a][0], f1 = kFace[a][1], f2 = kFace[a][2];
        // the longest of the three sides carries the line
        int s = f0, t = f1;
        double best = (qx[f1] - qx[f0]) * (qx[f1] - qx[f0]) + (qy[f1] - qy[f0]) * (qy[f1] - qy[f0]);
        const double l02 = (qx[f2] - qx[f0]) * (qx[f2] - qx[f0]) + (qy[f2] - qy[f0]) * (qy[f2] - qy[f0]);
        const double l12 = (qx[f2] - qx[f1]) * (qx[f2] - qx[f1]) + (qy[f2] - qy[f1]) * (qy[f2] - qy[f1]);
        if (l02 > best) { best = l02; s = f0; t = f2; }
        if (l12 > best) { best = l12; s = f1; t = f2; }
        const double dx = qx[t] - qx[s], dy = qy[t] - qy[s];
        const double side = dx * (qy[a] - qy[s]) - dy * (qx[a] - qx[s]);
        if (side == 0.0) return false;  // all four collinear
        const double sg = side > 0 ? 1.0 : -1.0;
        if (nw >= 2 || ng + nw >= 4) return false;
        const int o = 3 * (ng + nw);
        fp.c[o + 0] = sg * (dy * qx[s] - dx * qy[s]);
        fp.c[o + 1] = -sg * dy;
        fp.c[o + 2] = sg * dx;
        // outward normal (away from vertex a) = sg * (dy, -dx); pixels on the
        // line are kept iff it points to -u, or along the u axis to -v
        const double ou = sg * dy, ov = -sg * dx;
        if (ou < 0 || (ou == 0 && ov < 0)) ties |= (nw == 0 ? REC_TIE0 : REC_TIE1);
        ++nw;
    }
    fp.ng = ng;
    fp.nw = nw;
    fp.ties = ties;
    fp.cond = cond;
    return true;
}


// Counters of one lattice cube's setup.
struct CubeCounts {
    unsigned n_tets = 0, n_zero = 0, n_inv = 0, n_dets = 0, n_deg = 0;
};

// Setup of the six tetrahedra of lattice cube `cube`: gather and unwrap the
// corners, volume determinant with its FP64 fallback, footprint.  r[t] is the
// record of tetrahedron 6*cube + t (flags 0 when it can cover no pixel);
// want64[t] tells whether its footprint is to be rastered in FP64, with the
// FP64 coefficients in fp[t].
TESS_HD inline void setup_cube(const LatticeParams &L, const ViewParams &V, int64_t cube, TetRec r[6],
                               Footprint fp[6], bool want64[6], CubeCounts &cnt) {
    const int64_t i = cube % L.c[0];
    const int64_t rest = cube / L.c[0];
    const int64_t j = rest % L.c[1];
    const int64_t k = rest / L.c[1];
    // gather the eight corners (tracer id = i + d0 (j + d1 k))
    double X0[3] = {0, 0, 0};
    double e[8][3];
#pragma unroll
    for (int n = 0; n < 8; ++n) {
        int64_t ii = i + (n & 1), jj = j + ((n >> 1) & 1), kk = k + ((n >> 2) & 1);
        if (L.periodic) {
            if (ii == L.d[0]) ii = 0;
            if (jj == L.d[1]) jj = 0;
            if (kk == L.d[2]) kk = 0;
        }
        const int64_t id = ii + (int64_t)L.d[0] * (jj + (int64_t)L.d[1] * kk);
        const double p[3] = {(double)L.x[id], (double)L.y[id], (double)L.z[id]};
        if (n == 0) {
            X0[0] = p[0]; X0[1] = p[1]; X0[2] = p[2];
            e[0][0] = e[0][1] = e[0][2] = 0.0;
        } else {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                double d = p[a] - X0[a];  // exact: difference of two floats
                if (L.periodic) d -= L.box[a] * ceil(d / L.box[a] - 0.5);
                e[n][a] = d;
            }
        }
    }
    // projected corners in pixel units
    const double b0[3] = {X0[0] - V.center[0], X0[1] - V.center[1], X0[2] - V.center[2]};
    double PX0 = (V.rot[0] * b0[0] + V.rot[1] * b0[1] + V.rot[2] * b0[2] - V.u_left) * V.inv_du;
    double PY0 = (V.rot[3] * b0[0] + V.rot[4] * b0[1] + V.rot[5] * b0[2] - V.v_bottom) * V.inv_dv;
    if (V.wrap) {  // a periodic image: move corner 0 into the first period
        PX0 -= (double)V.W * floor(PX0 / (double)V.W);
        PY0 -= (double)V.H * floor(PY0 / (double)V.H);
    }
    double PX[8], PY[8];
#pragma unroll
    for (int n = 0; n < 8; ++n) {
        PX[n] = PX0 + (V.rot[0] * e[n][0] + V.rot[1] * e[n][1] + V.rot[2] * e[n][2]) * V.inv_du;
        PY[n] = PY0 + (V.rot[3] * e[n][0] + V.rot[4] * e[n][1] + V.rot[5] * e[n][2]) * V.inv_dv;
    }
#pragma unroll
    for (int t = 0; t < 6; ++t) {
        const int v0 = kTet[t][0], v1 = kTet[t][1], v2 = kTet[t][2], v3 = kTet[t][3];
        TetRec &R = r[t];
        R.h.bx = 0;
        R.h.by = 0;
        R.h.flags = 0;
        R.h.slot = kNoSlot;
#pragma unroll
        for (int g = 0; g < 12; ++g) R.c[g] = 0.f;
        want64[t] = false;
        // ---- volume determinant (Eq. Eqn:TetVolume), 6 V: FP32 with a forward
        // error bound, FP64 when the bound cannot certify it or it is small
        double a64[3], b64[3], c64[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            a64[q] = e[v1][q] - e[v0][q];
            b64[q] = e[v2][q] - e[v0][q];
            c64[q] = e[v3][q] - e[v0][q];
        }
        const float a[3] = {(float)a64[0], (float)a64[1], (float)a64[2]};
        const float b[3] = {(float)b64[0], (float)b64[1], (float)b64[2]};
        const float c[3] = {(float)c64[0], (float)c64[1], (float)c64[2]};
        const float p1 = b[1] * c[2], p2 = b[2] * c[1];
        const float p3 = b[2] * c[0], p4 = b[0] * c[2];
        const float p5 = b[0] * c[1], p6 = b[1] * c[0];
        const float d32 = a[0] * (p1 - p2) + a[1] * (p3 - p4) + a[2] * (p5 - p6);
        const float perm = fabsf(a[0]) * (fabsf(p1) + fabsf(p2)) + fabsf(a[1]) * (fabsf(p3) + fabsf(p4)) +
                           fabsf(a[2]) * (fabsf(p5) + fabsf(p6));
        const double ad = fabs((double)d32);
        const bool flagged = ad <= L.det_cond_k * 0x1p-24 * (double)perm ||
                             ad < 2.0 * 6.0 * L.det_v0_frac * L.v0;
        const double det6 = flagged ? det6_fp64(a64, b64, c64) : (double)d32;
        cnt.n_dets += flagged ? 1 : 0;
        if (det6 == 0.0) {
            ++cnt.n_zero;
            continue;
        }
        ++cnt.n_tets;
        cnt.n_inv += det6 > 0 ? 1 : 0;
        cnt.n_deg += fabs(det6) < 6.0 * L.det_v0_frac * L.v0 ? 1 : 0;
        // ---- screen footprint (FP64)
        const int vi[4] = {v0, v1, v2, v3};
        double xmin = PX[v0], xmax = PX[v0], ymin = PY[v0], ymax = PY[v0];
#pragma unroll
        for (int m = 1; m < 4; ++m) {
            xmin = fmin(xmin, PX[vi[m]]); xmax = fmax(xmax, PX[vi[m]]);
            ymin = fmin(ymin, PY[vi[m]]); ymax = fmax(ymax, PY[vi[m]]);
        }
        // pixel centres ix + 1/2 inside [xmin, xmax] (clamped far outside any image)
        const double lim = 1.0e8;
        int ix0 = (int)fmax(ceil(xmin - 0.5), -lim), ix1 = (int)fmin(floor(xmax - 0.5), lim);
        int iy0 = (int)fmax(ceil(ymin - 0.5), -lim), iy1 = (int)fmin(floor(ymax - 0.5), lim);
        if (!V.wrap) {
            ix0 = ix0 > 0 ? ix0 : 0;
            iy0 = iy0 > 0 ? iy0 : 0;
            ix1 = ix1 < V.W - 1 ? ix1 : V.W - 1;
            iy1 = iy1 < V.H - 1 ? iy1 : V.H - 1;
        }
        if (ix0 > ix1 || iy0 > iy1) continue;
        double qx[4], qy[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            qx[m] = PX[vi[m]] - (double)ix0;
            qy[m] = PY[vi[m]] - (double)iy0;
        }
        if (!footprint(qx, qy, V.mass_px, (double)(ix1 - ix0 + 1), (double)(iy1 - iy0 + 1), fp[t]))
            continue;
        R.h.bx = pack_range(ix0, ix1);
        R.h.by = pack_range(iy0, iy1);
        R.h.flags = (uint32_t)fp[t].ng | ((uint32_t)fp[t].nw << REC_NW_SHIFT) | fp[t].ties | REC_VALID;
#pragma unroll
        for (int g = 0; g < 12; ++g) R.c[g] = (float)fp[t].c[g];
        want64[t] = L.fp64_cond < 0.0 || fp[t].cond > L.fp64_cond;
    }
}

// ---------------------------------------------------------------- binning
// Tiles of one axis touched by the pixel range [b0, b1]: `count` tiles
// starting at `start`, taken modulo the tile count under wrap.
TESS_HD inline void axis_tiles(int b0, int b1, int n, int T, int ntiles, int wrap,
                                  int &start, int &count) {
    if (!wrap) {
        const int lo = max(b0, 0), hi = min(b1, n - 1);
        if (lo > hi) { start = 0; count = 0; return; }
        start = lo / T;
        count = hi / T - start + 1;
        return;
    }
    if (b1 - b0 + 1 >= n) { start = 0; count = ntiles; return; }
    const int a = imod(b0, n);
    const int b = a + (b1 - b0);
    if (b < n) { start = a / T; count = b / T - a / T + 1; return; }
    const int ta = a / T, tb = (b - n) / T;
    if (tb >= ta) { start = 0; count = ntiles; return; }
    start = ta;
    count = ntiles - ta + tb + 1;
}

// Offsets k (in units of the image size) for which tile pixels [t0, t1]
// shifted by k*n meet [b0, b1].
TESS_HD inline void axis_offsets(int t0, int t1, int b0, int b1, int n, int wrap, int &k0,
                                    int &k1) {
    if (!wrap) { k0 = 0; k1 = 0; return; }
    k0 = ceil_div(b0 - t1, n);
    k1 = floor_div(b1 - t0, n);
}

// Does some pixel centre of the rectangle [x0, x1] x [y0, y1] (pixel indices
// in the record's frame, already inside its bounding box) possibly get a
// nonzero value?  Conservative: rejects only when one function is negative
// at all four corner pixel centres; FP64-flagged footprints are never culled.
TESS_HD inline bool rect_may_cover(const TetRec &r, int x0, int x1, int y0, int y1) {
    if (r.h.flags & REC_FP64) return true;
    const float xa = (float)(x0 - range_lo(r.h.bx)) + 0.5f, xb = (float)(x1 - range_lo(r.h.bx)) + 0.5f;
    const float ya = (float)(y0 - range_lo(r.h.by)) + 0.5f, yb = (float)(y1 - range_lo(r.h.by)) + 0.5f;
    const int nf = (int)(r.h.flags & REC_NG_MASK) + (int)((r.h.flags >> REC_NW_SHIFT) & 3u);
    for (int g = 0; g < nf; ++g) {
        const float a = r.c[3 * g], b = r.c[3 * g + 1], c = r.c[3 * g + 2];
        const float mx = a + (b > 0 ? b * xb : b * xa) + (c > 0 ? c * yb : c * ya);
        // margin: values this small relative to the coefficients are rounding
        if (mx < -1e-5f * (fabsf(a) + fabsf(b) * fmaxf(fabsf(xa), fabsf(xb)) +
                           fabsf(c) * fmaxf(fabsf(ya), fabsf(yb))))
            return false;
    }
    return true;
}

TESS_HD inline bool tile_accept(const TetRec &r, int tx, int ty, const BinParams &B) {
    const int tx0 = tx * B.T, tx1 = min(tx0 + B.T, B.W) - 1;
    const int ty0 = ty * B.T, ty1 = min(ty0 + B.T, B.H) - 1;
    int kx0, kx1, ky0, ky1;
    axis_offsets(tx0, tx1, range_lo(r.h.bx), range_hi(r.h.bx), B.W, B.wrap, kx0, kx1);
    axis_offsets(ty0, ty1, range_lo(r.h.by), range_hi(r.h.by), B.H, B.wrap, ky0, ky1);
    for (int ky = ky0; ky <= ky1; ++ky)
        for (int kx = kx0; kx <= kx1; ++kx) {
            const int x0 = max(tx0 + kx * B.W, (int)range_lo(r.h.bx)), x1 = min(tx1 + kx * B.W, (int)range_hi(r.h.bx));
            const int y0 = max(ty0 + ky * B.H, (int)range_lo(r.h.by)), y1 = min(ty1 + ky * B.H, (int)range_hi(r.h.by));
            if (x0 > x1 || y0 > y1) continue;
            if (rect_may_cover(r, x0, x1, y0, y1)) return true;
        }
    return false;
}


// ----------------------------------------------------------------- raster
// Adds rho*dl of one footprint to the lane's L consecutive pixels; (x, y) is
// the first pixel centre in the record frame.  NG = 3 or 4, no walls.
template <typename R, int L, int NG, typename Sum>
TESS_HD inline void eval_fast(const R *c, R x, R y, Sum (&acc)[L]) {
    // g_q at the strip's first pixel centre, then one step of b_q per pixel
    R g[NG], b[NG];
#pragma unroll
    for (int q = 0; q < NG; ++q) {
        b[q] = c[3 * q + 1];
        g[q] = c[3 * q] + b[q] * x + c[3 * q + 2] * y;
    }
#pragma unroll
    for (int k = 0; k < L; ++k) {
        R m = fmin(g[0], fmin(g[1], g[2]));
        if (NG == 4) m = fmin(m, g[NG - 1]);
        acc[k] += (Sum)fmax(m, (R)0);
#pragma unroll
        for (int q = 0; q < NG; ++q) g[q] += b[q];
    }
}

// Any number of G functions plus walls with their tie bits.  With COUNT the
// number of covered pixels among the first `valid` ones is returned instead
// of accumulating.
template <typename R, int L, bool COUNT, typename Sum>
TESS_HD inline unsigned eval_general(const R *c, uint32_t flags, R x, R y, Sum (&acc)[L],
                                        int kmin, int kmax) {
    const int ng = (int)(flags & REC_NG_MASK);
    const int nw = (int)((flags >> REC_NW_SHIFT) & 3u);
    unsigned n = 0;
#pragma unroll
    for (int k = 0; k < L; ++k) {
        const R xk = x + (R)k;
        bool in = true;
        for (int q = 0; q < nw; ++q) {
            const R *w = c + 3 * (ng + q);
            const R wv = w[0] + w[1] * xk + w[2] * y;
            const bool tie = (flags & (q == 0 ? REC_TIE0 : REC_TIE1)) != 0;
            in = in && (wv > (R)0 || (wv == (R)0 && tie));
        }
        R m = (R)INFINITY;
        for (int q = 0; q < ng; ++q) m = fmin(m, c[3 * q] + c[3 * q + 1] * xk + c[3 * q + 2] * y);
        if (COUNT)
            n += (in && m > (R)0 && k >= kmin && k <= kmax) ? 1u : 0u;
        else if (in)
            acc[k] += (Sum)fmax(m, (R)0);
    }
    return n;
}

// Rare paths kept out of line so the hot loop keeps its registers: footprints
// with walls (edge-on faces), and FP64 footprints.
template <typename R, int L, typename Sum>
TESS_HD __attribute__((noinline)) void eval_slow(const R *c, uint32_t flags, R x, R y, Sum (&acc)[L]) {
    const int ng = (int)(flags & REC_NG_MASK);
    const bool walls = ((flags >> REC_NW_SHIFT) & 3u) != 0;
    if (!walls && ng == 4)
        eval_fast<R, L, 4>(c, x, y, acc);
    else if (!walls && ng == 3)
        eval_fast<R, L, 3>(c, x, y, acc);
    else
        eval_general<R, L, false>(c, flags, x, y, acc, 0, L - 1);
}

template <typename R, int L, typename Sum>
TESS_HD inline void eval_any(const R *c, uint32_t flags, R x, R y, Sum (&acc)[L]) {
    const int ng = (int)(flags & REC_NG_MASK);
    const bool walls = ((flags >> REC_NW_SHIFT) & 3u) != 0;
    if (!walls && ng == 4)
        eval_fast<R, L, 4>(c, x, y, acc);
    else if (!walls && ng == 3)
        eval_fast<R, L, 3>(c, x, y, acc);
    else
        eval_slow<R, L>(c, flags, x, y, acc);
}

// Candidate tiles of one record: tx = (sx + s % cx) mod ntx, ty = (sy + s / cx)
// mod nty for s < count = cx * cy.
struct TileRange {
    int sx, cx, sy, cy, count;
};

TESS_HD inline TileRange tet_tiles(const TetRec &r, const BinParams &B) {
    TileRange t;
    axis_tiles(range_lo(r.h.bx), range_hi(r.h.bx), B.W, B.T, B.ntx, B.wrap, t.sx, t.cx);
    axis_tiles(range_lo(r.h.by), range_hi(r.h.by), B.H, B.T, B.nty, B.wrap, t.sy, t.cy);
    t.count = t.cx * t.cy;
    return t;
}

// Candidate s of the record: its tile index, and whether the footprint may
// cover a pixel centre there.
TESS_HD inline bool tet_tile(const TetRec &r, const BinParams &B, const TileRange &t, int s, int &tile) {
    int tx = t.sx + s % t.cx, ty = t.sy + s / t.cx;
    if (tx >= B.ntx) tx -= B.ntx;
    if (ty >= B.nty) ty -= B.nty;
    tile = ty * B.ntx + tx;
    return tile_accept(r, tx, ty, B);
}

// Accumulator of one lane's L pixels: FP32 block sums folded into FP64, and
// FP64 terms added to the FP64 part directly.
constexpr int kFlushEvery = 32;  // FP32 partial sums are folded into FP64 this often

template <int L>
struct Acc {
    float s[L];
    double d[L];
    TESS_HD void zero() {
#pragma unroll
        for (int k = 0; k < L; ++k) { s[k] = 0.f; d[k] = 0.0; }
    }
    TESS_HD void flush() {
#pragma unroll
        for (int k = 0; k < L; ++k) { d[k] += (double)s[k]; s[k] = 0.f; }
    }
};


// Geometry of one raster lane: the L-pixel strip of lane `tid` of the T x T
// tile `tile` (T / L lanes per row).
struct LaneGeom {
    int tile_x0, tile_x1, tile_y0, tile_y1;  // tile pixels (inclusive, clipped to the image)
    int px0, py;                             // first pixel of the strip
    int wy0, wy1;                            // rows of the lane's wavefront
    int valid;                               // strip pixels inside the image
    bool live;                               // some strip pixel inside the image
};

template <int T, int L>
TESS_HD inline LaneGeom lane_geom(uint32_t tile, const BinParams &B, int tid) {
    constexpr int SPR = T / L;                 // strips per row
    constexpr int RPW = 64 / SPR;              // rows per wavefront
    LaneGeom g;
    const int tx = (int)(tile % (uint32_t)B.ntx), ty = (int)(tile / (uint32_t)B.ntx);
    const int row = tid / SPR, strip = tid % SPR;
    g.tile_x0 = tx * T;
    g.tile_y0 = ty * T;
    g.tile_x1 = (g.tile_x0 + T < B.W ? g.tile_x0 + T : B.W) - 1;
    g.tile_y1 = (g.tile_y0 + T < B.H ? g.tile_y0 + T : B.H) - 1;
    g.px0 = g.tile_x0 + strip * L;
    g.py = g.tile_y0 + row;
    g.wy0 = g.tile_y0 + (tid / 64) * RPW;
    g.wy1 = g.wy0 + RPW - 1;
    // lanes whose pixels lie beyond the image (ragged last tiles) stay idle
    g.live = g.py <= g.tile_y1 && g.px0 <= g.tile_x1;
    g.valid = L < g.tile_x1 - g.px0 + 1 ? L : g.tile_x1 - g.px0 + 1;
    return g;
}

// Periodic offsets of a record against a tile: a box inside the image needs
// none (fast path), otherwise the general division.
TESS_HD inline void rec_offsets(int t0, int t1, int b0, int b1, int n, int wrap, int &k0, int &k1) {
    if (!wrap || (b0 >= 0 && b1 < n)) {
        k0 = 0;
        k1 = 0;
        return;
    }
    axis_offsets(t0, t1, b0, b1, n, wrap, k0, k1);
}

// Adds one record's footprint to the lane's strip (every periodic offset that
// meets the tile).  c64: the record's FP64 coefficients when REC_FP64.
template <int L, bool COUNT>
TESS_HD inline void raster_record(const TetRec &r, const double *c64, const BinParams &B,
                                  const LaneGeom &g, Acc<L> &acc, unsigned &frags, unsigned &frags4) {
    const bool f64 = (r.h.flags & REC_FP64) != 0;
    const int bx0 = range_lo(r.h.bx), bx1 = range_hi(r.h.bx);
    const int by0 = range_lo(r.h.by), by1 = range_hi(r.h.by);
    int kx0, kx1, ky0, ky1;
    rec_offsets(g.tile_x0, g.tile_x1, bx0, bx1, B.W, B.wrap, kx0, kx1);
    rec_offsets(g.tile_y0, g.tile_y1, by0, by1, B.H, B.wrap, ky0, ky1);
    for (int ky = ky0; ky <= ky1; ++ky) {
        // wavefront-uniform row test
        if (g.wy1 + ky * B.H < by0 || g.wy0 + ky * B.H > by1) continue;
        for (int kx = kx0; kx <= kx1; ++kx) {
            const int gy = g.py + ky * B.H;
            const int gx0 = g.px0 + kx * B.W;
            if (!g.live || gy < by0 || gy > by1 || gx0 + L - 1 < bx0 || gx0 > bx1) continue;
            unsigned nf = 0;
            const int kmin = bx0 - gx0 > 0 ? bx0 - gx0 : 0;
            const int kmax = g.valid - 1 < bx1 - gx0 ? g.valid - 1 : bx1 - gx0;
            if (!f64) {
                const float x = (float)(gx0 - bx0) + 0.5f;
                const float y = (float)(gy - by0) + 0.5f;
                eval_any<float, L>(r.c, r.h.flags, x, y, acc.s);
                if (COUNT) nf = eval_general<float, L, true>(r.c, r.h.flags, x, y, acc.s, kmin, kmax);
            } else {
                const double x = (double)(gx0 - bx0) + 0.5;
                const double y = (double)(gy - by0) + 0.5;
                eval_slow<double, L>(c64, r.h.flags, x, y, acc.d);
                if (COUNT) nf = eval_general<double, L, true>(c64, r.h.flags, x, y, acc.d, kmin, kmax);
            }
            frags += nf;
            if ((r.h.flags & REC_NG_MASK) == 4) frags4 += nf;
        }
    }
}

// The work of one raster lane over a work item's list, in list order (the
// kernel does the same with records staged through LDS).
template <int T, int L, bool COUNT>
TESS_HD inline void raster_lane(const TetRec *rec, const Coef64 *coef64, uint32_t coef64_cap,
                                const uint32_t *pairs, const WorkItem &it, const BinParams &B, int tid,
                                Acc<L> &acc, unsigned &frags, unsigned &frags4) {
    const LaneGeom g = lane_geom<T, L>(it.tile, B, tid);
    acc.zero();
    frags = frags4 = 0;
    int since_flush = 0;
    for (uint32_t e = 0; e < it.count; ++e) {
        const uint32_t id = pairs[it.first + e];
        if (id < B.ntet) {
            const TetRec r = rec[id];
            const bool f64 = (r.h.flags & REC_FP64) != 0;
            if (!f64 || r.h.slot < coef64_cap)
                raster_record<L, COUNT>(r, f64 ? coef64[r.h.slot].c : nullptr, B, g, acc, frags, frags4);
        }
        if (++since_flush == kFlushEvery) {
            acc.flush();
            since_flush = 0;
        }
    }
    acc.flush();
}

}  // namespace tess
