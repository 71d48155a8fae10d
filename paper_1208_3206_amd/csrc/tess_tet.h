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

constexpr double kPi = 3.14159265358979323846;

// Mesh edges.  The table's tetrahedra fit together across cubes (every face
// diagonal runs the same way on opposite faces), so each lattice vertex owns
// seven edges, to cube corners 1, 2 and 4 from corner 0, the face diagonals
// 1-2, 1-4 and 2-4, and the body diagonal 3-4 of the cube that has the vertex
// as corner 0.  Edge tau runs between corners kEdgeEnds[tau][0] and [1];
// the tetrahedra holding it are tetrahedron t of the cube moved by (dx, dy,
// dz) in {-1, 0}^3, where it is local edge e (local edges of kTet[t]: vertex
// pairs 01, 02, 03, 12, 13, 23).  36 entries: each of a cube's 6 x 6
// tetrahedron edges once.
constexpr int kEdgeEnds[7][2] = {{0, 1}, {0, 2}, {0, 4}, {1, 2}, {1, 4}, {2, 4}, {3, 4}};
struct EdgeUse {
    int8_t dx, dy, dz, t, e;
};
constexpr int kEdgeFirst[8] = {0, 6, 12, 16, 20, 26, 32, 36};
constexpr EdgeUse kEdgeUse[36] = {
    {0, -1, -1, 5, 4}, {0, -1, 0, 1, 1}, {0, -1, 0, 4, 0}, {0, 0, -1, 2, 4}, {0, 0, -1, 3, 5}, {0, 0, 0, 0, 0},
    {-1, 0, -1, 5, 3}, {-1, 0, 0, 1, 0}, {-1, 0, 0, 2, 1}, {0, 0, -1, 3, 4}, {0, 0, -1, 4, 5}, {0, 0, 0, 0, 3},
    {-1, -1, 0, 5, 0}, {-1, 0, 0, 2, 3}, {0, -1, 0, 4, 3}, {0, 0, 0, 0, 4},
    {0, 0, -1, 3, 3}, {0, 0, -1, 5, 5}, {0, 0, 0, 0, 1}, {0, 0, 0, 1, 3},
    {0, -1, 0, 3, 0}, {0, -1, 0, 4, 1}, {0, -1, 0, 5, 2}, {0, 0, 0, 0, 2}, {0, 0, 0, 1, 4}, {0, 0, 0, 2, 5},
    {-1, 0, 0, 2, 0}, {-1, 0, 0, 3, 1}, {-1, 0, 0, 5, 1}, {0, 0, 0, 0, 5}, {0, 0, 0, 1, 5}, {0, 0, 0, 4, 4},
    {0, 0, 0, 1, 2}, {0, 0, 0, 2, 2}, {0, 0, 0, 3, 2}, {0, 0, 0, 4, 2}};

// The inverse of kEdgeUse: local edge e of tetrahedron t of cube c is entry
// u of edge kind tau of the vertex at c + (ox, oy, oz), o = -d in {0, 1}^3
// (a corner of c).  Setup writes each tetrahedron's slope changes into these
// slots, 36 per vertex in the order of kEdgeUse and stored slot-major (slot u
// of vertex w at u * nvert + w), so that both the writes of neighbouring
// cubes and the reads of neighbouring vertices are contiguous.
struct EdgeSlot {
    int8_t u, ox, oy, oz;
};
struct EdgeSlots {
    EdgeSlot s[6][6];
};
constexpr EdgeSlots make_edge_slots() {
    EdgeSlots T{};
    for (int u = 0; u < 36; ++u) {
        const EdgeUse U = kEdgeUse[u];
        T.s[U.t][U.e] = EdgeSlot{(int8_t)u, (int8_t)-U.dx, (int8_t)-U.dy, (int8_t)-U.dz};
    }
    return T;
}
constexpr EdgeSlots kEdgeSlots = make_edge_slots();

// local edge index of the tetrahedron vertex pair (u, v), u != v
TESS_HD inline int local_edge(int u, int v) {
    const int a = u < v ? u : v, b = u < v ? v : u;
    return a == 0 ? b - 1 : (a == 1 ? b + 1 : 5);
}


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
// floor(a / b) for b > 0 and |a|, b below 2^22 (pixel and tile sizes): the
// FP32 quotient from the reciprocal, then one correction step makes it exact
// (the estimate is within one of the quotient), about a fifth of the cost
// of an integer division on the GPU
TESS_HD inline int floor_div_r(int a, int b, float rb) {  // rb: 1/b within a few ulp
    int q = (int)floorf((float)a * rb);
    const int r = a - q * b;
    if (r < 0) --q;
    else if (r >= b) ++q;
    return q;
}
TESS_HD inline int floor_div(int a, int b) {
#ifdef __HIP_DEVICE_COMPILE__
    return floor_div_r(a, b, __builtin_amdgcn_rcpf((float)b));
#else
    return floor_div_r(a, b, 1.0f / (float)b);
#endif
}
TESS_HD inline int ceil_div(int a, int b) {  // b > 0
    return -floor_div(-a, b);
}
TESS_HD inline int imod(int a, int m) {  // in [0, m), m > 0 (as floor_div)
    return a - m * floor_div(a, m);
}
// 1/s to within a few ulp: the hardware estimate refined by one Newton step
// (the host build divides).
TESS_HD inline double fast_rcp(double s) {
#ifdef __HIP_DEVICE_COMPILE__
    const double r = __builtin_amdgcn_rcp(s);
    return fma(fma(-s, r, 1.0), r, r);
#else
    return 1.0 / s;
#endif
}


// Volume determinant (times 6) in FP64, evaluated term by term without
// contraction so that an exact zero is decided the same way as by a plain
// left-to-right FP64 evaluation of Eq. Eqn:TetVolume.
TESS_HD inline double det6_fp64(const double a[3], const double b[3], const double c[3]) {
#pragma clang fp contract(off)
    double cx = b[1] * c[2] - b[2] * c[1];
    double cy = b[2] * c[0] - b[0] * c[2];
    double cz = b[0] * c[1] - b[1] * c[0];
    return a[0] * cx + a[1] * cy + a[2] * cz;
}

// ------------------------------------------------------ footprint setup
struct Footprint {
    double c[12];
    int ei[4], ej[4];  // tetrahedron vertices of silhouette edge g
    int ng, nw;
    uint32_t ties;
};

// Builds the G functions and walls of one tetrahedron from its projected
// vertices q (pixel units, relative to the record origin).  Returns false
// when the projection has zero area (no pixel can receive anything).
TESS_HD inline bool footprint(const double qx[4], const double qy[4], double mass_px, Footprint &fp) {
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
    int ng = 0, nw = 0;
    uint32_t ties = 0;
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
            // slot ng, by compile-time slots (an indexed store would put the
            // arrays in scratch memory)
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (k == ng) {
                    fp.c[3 * k + 0] = aa;
                    fp.c[3 * k + 1] = bb;
                    fp.c[3 * k + 2] = cc;
                    fp.ei[k] = E.i;
                    fp.ej[k] = E.j;
                }
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
        const double w0 = sg * (dy * qx[s] - dx * qy[s]), w1 = -sg * dy, w2 = sg * dx;
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (k == ng + nw) {
                fp.c[3 * k + 0] = w0;
                fp.c[3 * k + 1] = w1;
                fp.c[3 * k + 2] = w2;
            }
        // outward normal (away from vertex a) = sg * (dy, -dx); pixels on the
        // line are kept iff it points to -u, or along the u axis to -v
        const double ou = sg * dy, ov = -sg * dx;
        if (ou < 0 || (ou == 0 && ov < 0)) ties |= (nw == 0 ? REC_TIE0 : REC_TIE1);
        ++nw;
    }
    fp.ng = ng;
    fp.nw = nw;
    fp.ties = ties;
    return true;
}


// Crease form of a footprint without walls.  The pyramid's creases are the
// silhouette edges and the ridges from the apex to the silhouette vertices:
// the apex is the vertex inside the silhouette triangle (three silhouette
// edges) or the crossing of the quadrilateral's diagonals (four).  Along a
// pixel row the footprint's slope jumps by |b| at a silhouette edge and by
// -|b_k-1 - b_k| at the ridge to V_k, with b the x slopes of the faces over
// the silhouette edges.  Returns false if the edges do not close a cycle.
// The silhouette edges as a cycle: vertices V_0..V_m-1 and, for the cyclic
// edge (V_k, V_k+1), its G function Lk[k].  False if they close no cycle.
TESS_HD inline bool crease_cycle(const Footprint &fp, int V[4], int Lk[4]) {
    const int m = fp.ng;
    if (m != 3 && m != 4) return false;
    V[0] = fp.ei[0]; V[1] = fp.ej[0]; V[2] = 0; V[3] = 0;
    Lk[0] = 0; Lk[1] = 0; Lk[2] = 0; Lk[3] = 0;
#pragma unroll
    for (int k = 1; k < 4; ++k) {
        if (k >= m) break;
        int found = -1, next = -1;
#pragma unroll
        for (int l = 1; l < 4; ++l) {
            if (l >= m || l == Lk[k - 1] || found >= 0) continue;
            if (fp.ei[l] == V[k]) { found = l; next = fp.ej[l]; }
            else if (fp.ej[l] == V[k]) { found = l; next = fp.ei[l]; }
        }
        if (found < 0) return false;
        Lk[k] = found;
        if (k + 1 < m) V[k + 1] = next;
        else if (next != V[0]) return false;
    }
    return true;
}

TESS_HD inline bool crease_payload(const double qx[4], const double qy[4], const Footprint &fp,
                                   double out[14]) {
    const int m = fp.ng;
    int V[4], Lk[4];  // silhouette edge g of cyclic edge (V_k, V_k+1)
    if (!crease_cycle(fp, V, Lk)) return false;
    double vx[4], vy[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int v = V[k];
        vx[k] = v == 0 ? qx[0] : v == 1 ? qx[1] : v == 2 ? qx[2] : qx[3];
        vy[k] = v == 0 ? qy[0] : v == 1 ? qy[1] : v == 2 ? qy[2] : qy[3];
    }
    double ax, ay;
    if (m == 3) {
        const int p = 6 - V[0] - V[1] - V[2];  // the vertex on no silhouette edge
        ax = p == 0 ? qx[0] : p == 1 ? qx[1] : p == 2 ? qx[2] : qx[3];
        ay = p == 0 ? qy[0] : p == 1 ? qy[1] : p == 2 ? qy[2] : qy[3];
    } else {
        const double d1x = vx[2] - vx[0], d1y = vy[2] - vy[0];
        const double d2x = vx[3] - vx[1], d2y = vy[3] - vy[1];
        const double den = d1x * d2y - d1y * d2x;
        if (den == 0.0) return false;
        const double t = ((vx[1] - vx[0]) * d2y - (vy[1] - vy[0]) * d2x) / den;
        ax = vx[0] + t * d1x;
        ay = vy[0] + t * d1y;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const bool real = k < m;
        const int g = Lk[k];
        out[k] = real ? vx[k] : 0.0;
        out[4 + k] = real ? vy[k] : 0.0;
        out[10 + k] = real ? (g == 0 ? fp.c[1] : g == 1 ? fp.c[4] : g == 2 ? fp.c[7] : fp.c[10]) : 0.0;
    }
    out[8] = ax;
    out[9] = ay;
    return true;
}

// The pyramid's creases by tetrahedron edge (the edge form): every crease
// lies on the projection of one of the six edges (silhouette edges, the
// ridges of a triangular silhouette, the diagonals of a quadrilateral one),
// so the footprint is the sum over the six local edges e of a slope change
// D[e] along the edge's projection.  sil gets 2 bits per local edge: 1 for an
// entering silhouette edge (b > 0), 2 for a leaving one.  D[e] as in the
// crease form: |b| on the silhouette, -|b_k-1 - b_k| on the ridge to V_k; the
// two halves of a diagonal have the same change (both are the difference of
// the two faces meeting along it), and the mean of the two is taken.
TESS_HD inline bool crease_kinks(const double qx[4], const double qy[4], const Footprint &fp, double D[6],
                                 uint32_t &sil) {
    int V[4], Lk[4];
    if (!crease_cycle(fp, V, Lk)) return false;
    const int m = fp.ng;
    if (m == 4) {  // the diagonals must cross, as the crease form requires
        auto px = [&](int v) { return v == 0 ? qx[0] : v == 1 ? qx[1] : v == 2 ? qx[2] : qx[3]; };
        auto py = [&](int v) { return v == 0 ? qy[0] : v == 1 ? qy[1] : v == 2 ? qy[2] : qy[3]; };
        const double den = (px(V[2]) - px(V[0])) * (py(V[3]) - py(V[1])) -
                           (py(V[2]) - py(V[0])) * (px(V[3]) - px(V[1]));
        if (den == 0.0) return false;
    }
    double b[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int g = Lk[k];
        b[k] = k < m ? (g == 0 ? fp.c[1] : g == 1 ? fp.c[4] : g == 2 ? fp.c[7] : fp.c[10]) : 0.0;
    }
#pragma unroll
    for (int e = 0; e < 6; ++e) D[e] = 0.0;
    sil = 0u;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (k >= m) continue;
        const int k1 = k + 1 < m ? k + 1 : 0;
        const int e = local_edge(V[k], V[k1]);
#pragma unroll
        for (int f = 0; f < 6; ++f)
            if (f == e) D[f] = fabs(b[k]);
        sil |= (b[k] > 0.0 ? 1u : 2u) << (2 * e);
    }
    if (m == 3) {
        const int p = 6 - V[0] - V[1] - V[2];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int e = local_edge(p, V[k]);
            const double r = -fabs(b[k > 0 ? k - 1 : 2] - b[k]);
#pragma unroll
            for (int f = 0; f < 6; ++f)
                if (f == e) D[f] = r;
        }
    } else {
        const int e02 = local_edge(V[0], V[2]), e13 = local_edge(V[1], V[3]);
        const double r02 = -0.5 * (fabs(b[3] - b[0]) + fabs(b[1] - b[2]));
        const double r13 = -0.5 * (fabs(b[0] - b[1]) + fabs(b[2] - b[3]));
#pragma unroll
        for (int f = 0; f < 6; ++f) {
            if (f == e02) D[f] = r02;
            if (f == e13) D[f] = r13;
        }
    }
    return true;
}

// Row profile of a crease-form payload, kept in the record head for the
// binning's work classes: for the silhouette vertices V_0..V_3 and the apex,
// the first record row whose centre lies at or above the point (a crease
// from P to Q covers rows [min, max) of the two), shifted right by s so that
// the footprint's height fits 5 bits; 5 bits each from bit 0, s in bits 25-29.
TESS_HD inline uint32_t crease_profile(const double cf[14], int height) {
    int sh = 0;
    while (sh < 26 && (height >> sh) > 31) ++sh;
    uint32_t p = (uint32_t)sh << 25;
#pragma unroll
    for (int v = 0; v < 5; ++v) {
        const double y = v < 4 ? cf[4 + v] : cf[9];
        const int yb = (int)fmin(fmax(ceil(y - 0.5), 0.0), (double)height);
        p |= (uint32_t)min(yb >> sh, 31) << (5 * v);
    }
    return p;
}

// Face form of a tetrahedron (views with a depth slab): per face g its depth
// plane t = c0 + c1 x + c2 y through the projected vertices (q, T: pixel
// coordinates relative to the record origin, world depths), marked front
// when the opposite vertex lies behind it (the ray enters there) and back
// otherwise; a face seen edge-on is a wall, stored and tied as in the line
// form. qv is the projected value q. Returns false when the tetrahedron lies
// outside the slab or its projection is degenerate.
TESS_HD inline bool face_payload(const double qx[4], const double qy[4], const double T[4], double s0,
                                 double s1, double qv, double out[14], uint32_t &flags) {
    if (fmax(fmax(T[0], T[1]), fmax(T[2], T[3])) <= s0 || fmin(fmin(T[0], T[1]), fmin(T[2], T[3])) >= s1)
        return false;
    uint32_t fl = 0;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const int b = kFace[a][0], c = kFace[a][1], d = kFace[a][2];
        const double ex = qx[c] - qx[b], ey = qy[c] - qy[b];
        const double fx = qx[d] - qx[b], fy = qy[d] - qy[b];
        const double D = ex * fy - ey * fx;
        if (D == 0.0) {
            // the longest of the three sides carries the wall's line
            int s = b, t = c;
            double best = ex * ex + ey * ey;
            const double lbd = fx * fx + fy * fy;
            const double lcd = (qx[d] - qx[c]) * (qx[d] - qx[c]) + (qy[d] - qy[c]) * (qy[d] - qy[c]);
            if (lbd > best) { best = lbd; s = b; t = d; }
            if (lcd > best) { best = lcd; s = c; t = d; }
            const double dx = qx[t] - qx[s], dy = qy[t] - qy[s];
            const double side = dx * (qy[a] - qy[s]) - dy * (qx[a] - qx[s]);
            if (side == 0.0) return false;  // all four collinear
            const double sg = side > 0 ? 1.0 : -1.0;
            out[3 * a + 0] = sg * (dy * qx[s] - dx * qy[s]);
            out[3 * a + 1] = -sg * dy;
            out[3 * a + 2] = sg * dx;
            const double ou = sg * dy, ov = -sg * dx;
            if (ou < 0 || (ou == 0 && ov < 0)) fl |= 1u << (REC_FACE_TIE_SHIFT + a);
            fl |= REC_FACE_WALL << (REC_FACE_TYPE_SHIFT + 2 * a);
        } else {
            const double et = T[c] - T[b], ft = T[d] - T[b];
            const double c1 = (et * fy - ey * ft) / D, c2 = (ex * ft - et * fx) / D;
            const double c0 = T[b] - c1 * qx[b] - c2 * qy[b];
            const double side = T[a] - (c0 + c1 * qx[a] + c2 * qy[a]);
            if (side == 0.0) return false;
            out[3 * a + 0] = c0;
            out[3 * a + 1] = c1;
            out[3 * a + 2] = c2;
            fl |= (side > 0.0 ? REC_FACE_FRONT : REC_FACE_BACK) << (REC_FACE_TYPE_SHIFT + 2 * a);
        }
    }
    out[12] = qv;
    out[13] = 0.0;
    flags = fl;
    return true;
}

// Counters of one lattice cube's setup.
struct CubeCounts {
    unsigned n_tets = 0, n_zero = 0, n_inv = 0, n_dets = 0, n_deg = 0;
};

// 6 V of the tetrahedron on cube corners v0..v3 (offsets e from corner 0),
// Eq. Eqn:TetVolume: FP32 with a forward error bound, FP64 when the bound
// cannot certify it or it is small (flagged).
TESS_HD inline double tet_det6(const LatticeParams &L, const double e[8][3], int v0, int v1, int v2, int v3,
                               bool &flagged);
// The same from the tetrahedron's own four corner offsets ev.
TESS_HD inline double tet_det6(const LatticeParams &L, const double ev[4][3], bool &flagged) {
    double a64[3], b64[3], c64[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        a64[q] = ev[1][q] - ev[0][q];
        b64[q] = ev[2][q] - ev[0][q];
        c64[q] = ev[3][q] - ev[0][q];
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
    flagged = L.det_cond_k < 0.0 || ad <= L.det_cond_k * 0x1p-24 * (double)perm ||
              ad < 2.0 * 6.0 * L.det_v0_frac * L.v0;
    return flagged ? det6_fp64(a64, b64, c64) : (double)d32;
}
TESS_HD inline double tet_det6(const LatticeParams &L, const double e[8][3], int v0, int v1, int v2, int v3,
                               bool &flagged) {
    const double ev[4][3] = {{e[v0][0], e[v0][1], e[v0][2]}, {e[v1][0], e[v1][1], e[v1][2]},
                             {e[v2][0], e[v2][1], e[v2][2]}, {e[v3][0], e[v3][1], e[v3][2]}};
    return tet_det6(L, ev, flagged);
}

// Tetrahedron T's corners from the cube's arrays, by constant index.
template <int T>
TESS_HD inline void tet_corners_t(const double e[8][3], const double PX[8], const double PY[8], double ev[4][3],
                                  double pxv[4], double pyv[4]) {
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        ev[m][0] = e[kTet[T][m]][0];
        ev[m][1] = e[kTet[T][m]][1];
        ev[m][2] = e[kTet[T][m]][2];
        pxv[m] = PX[kTet[T][m]];
        pyv[m] = PY[kTet[T][m]];
    }
}
// The same for a tetrahedron t known only at run time: a switch (one
// branch when t is the same across the wavefront) instead of an array
// indexed by t, which the compiler would put in scratch memory.
TESS_HD inline void tet_corners(int t, const double e[8][3], const double PX[8], const double PY[8],
                                double ev[4][3], double pxv[4], double pyv[4]) {
    switch (t) {
        case 0: tet_corners_t<0>(e, PX, PY, ev, pxv, pyv); break;
        case 1: tet_corners_t<1>(e, PX, PY, ev, pxv, pyv); break;
        case 2: tet_corners_t<2>(e, PX, PY, ev, pxv, pyv); break;
        case 3: tet_corners_t<3>(e, PX, PY, ev, pxv, pyv); break;
        case 4: tet_corners_t<4>(e, PX, PY, ev, pxv, pyv); break;
        default: tet_corners_t<5>(e, PX, PY, ev, pxv, pyv); break;
    }
}

// The setup's counts for one tetrahedron of determinant det6.
TESS_HD inline void count_tet(const LatticeParams &L, double det6, bool flagged, CubeCounts &cnt) {
    cnt.n_dets += flagged ? 1 : 0;
    if (det6 == 0.0) {
        ++cnt.n_zero;
        return;
    }
    ++cnt.n_tets;
    cnt.n_inv += det6 > 0 ? 1 : 0;
    cnt.n_deg += fabs(det6) < 6.0 * L.det_v0_frac * L.v0 ? 1 : 0;
}

// The eight corners of a lattice cube: corner 0's position X0 and every
// corner's offset e[n] from it, unwrapped to the nearest periodic image.
// Returns true when some corner was moved by a box length.
// Lattice coordinates (i, j, k) of cube `cube` = i + c0 (j + c1 k): in
// 32-bit arithmetic (two divisions) below 2^31 cubes.
TESS_HD inline void cube_ijk(const LatticeParams &L, int64_t cube, int64_t &i, int64_t &j, int64_t &k) {
    if (L.ncubes <= 0x7fffffff) {
        const uint32_t c = (uint32_t)cube, c0 = (uint32_t)L.c[0], c1 = (uint32_t)L.c[1];
        const uint32_t r = c / c0, kk = r / c1;
        i = (int64_t)(c - r * c0);
        j = (int64_t)(r - kk * c1);
        k = (int64_t)kk;
    } else {
        const int64_t r = cube / L.c[0];
        i = cube - r * L.c[0];
        k = r / L.c[1];
        j = r - k * L.c[1];
    }
}

TESS_HD inline bool cube_corners(const LatticeParams &L, int64_t cube, double X0[3], double e[8][3]) {
    bool moved = false;
    int64_t i, j, k;
    cube_ijk(L, cube, i, j, k);
    // gather the eight corners (tracer id = i + d0 (j + d1 k))
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
                if (L.periodic) {
                    const double sh = ceil(d / L.box[a] - 0.5);
                    moved = moved || sh != 0.0;
                    d -= L.box[a] * sh;
                }
                e[n][a] = d;
            }
        }
    }
    return moved;
}

// Sum over the cube's six tetrahedra of q |V|, q = rho^qpow, rho = m / |V|:
// the integral of the projected value over the image when every tetrahedron
// is in view. Determinants in FP64, as setup_cube takes them for qpow != 1.
TESS_HD inline double cube_qvol(const LatticeParams &L, const ViewParams &V, int64_t cube) {
    double X0[3], e[8][3];
    cube_corners(L, cube, X0, e);
    double sum = 0.0;
#pragma unroll
    for (int t = 0; t < 6; ++t) {
        const int v0 = kTet[t][0], v1 = kTet[t][1], v2 = kTet[t][2], v3 = kTet[t][3];
        double a[3], b[3], c[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            a[q] = e[v1][q] - e[v0][q];
            b[q] = e[v2][q] - e[v0][q];
            c[q] = e[v3][q] - e[v0][q];
        }
        const double vol = fabs(det6_fp64(a, b, c)) / 6.0;
        if (vol == 0.0) continue;
        sum += V.qpow == 0 ? vol : (V.qpow == 1 ? L.tet_mass : L.tet_mass * L.tet_mass / vol);
    }
    return sum;
}

// Pixel x of lattice vertex `id` in its own frame (the frame of the cube
// that has it as corner 0; under wrap, moved into the first period), the
// same arithmetic in setup and in the edge records.
TESS_HD inline double vertex_px(const LatticeParams &L, const ViewParams &V, int64_t id) {
    const double b0[3] = {(double)L.x[id] - V.center[0], (double)L.y[id] - V.center[1],
                          (double)L.z[id] - V.center[2]};
    double px = (V.rot[0] * b0[0] + V.rot[1] * b0[1] + V.rot[2] * b0[2] - V.u_left) * V.inv_du;
    if (V.wrap) px -= (double)V.W * floor(px * V.inv_W);
    return px;
}

// Edge form, the common case of one tetrahedron taken directly: its six
// slope changes kd (the crease form's, as crease_kinks gives them), the
// silhouette kinds sil (2 bits per local edge) and the period offsets shf (2
// bits per local edge, s + 1), with the counts.  The pyramid's creases
// follow from the silhouette set alone: a silhouette edge (i, j) changes the
// row slope by |b|, b the x slope of its face function (footprint's K
// times -dy); any other edge is a ridge or a diagonal, whose change is
// -|b(v, k) - b(v, l)| at an end v whose edges to the other two vertices k,
// l are both silhouette edges (one end for a ridge of a triangular
// silhouette, both ends for a diagonal of a quadrilateral one, averaged).
// Returns -1, having counted nothing, when the tetrahedron needs the
// general setup: a face seen edge-on, a silhouette set that is neither a
// triangle nor a quadrilateral, crossing diagonals not found, or a period
// or margin test that fails; 0 (zeros) when it has no volume or covers no
// pixel centre; 8 when its footprint is steep along x, past the crease
// form's bound: it then keeps its own record in the line form, returned in
// own; else its number of silhouette edges.
template <typename OwnSink>
TESS_HD inline int edge_tet_fast(const LatticeParams &L, const ViewParams &V, int t, const double e[8][3],
                                 const double PX[8], const double PY[8], double crease_bmax, bool same_frame,
                                 uint32_t qpack, double kd[6], uint32_t &sil, uint32_t &shf, OwnSink &&own_sink,
                                 CubeCounts &cnt) {
    const int v0 = kTet[t][0], v1 = kTet[t][1], v2 = kTet[t][2], v3 = kTet[t][3];
    bool flagged;
    const double det6 = tet_det6(L, e, v0, v1, v2, v3, flagged);
    if (det6 == 0.0) {
        count_tet(L, det6, flagged, cnt);
        return 0;
    }
    const int vi[4] = {v0, v1, v2, v3};
    double xmin = PX[v0], xmax = PX[v0], ymin = PY[v0], ymax = PY[v0];
#pragma unroll
    for (int m = 1; m < 4; ++m) {
        xmin = fmin(xmin, PX[vi[m]]); xmax = fmax(xmax, PX[vi[m]]);
        ymin = fmin(ymin, PY[vi[m]]); ymax = fmax(ymax, PY[vi[m]]);
    }
    const double lim = 1.0e8;
    int ix0 = (int)fmax(ceil(xmin - 0.5), -lim), ix1 = (int)fmin(floor(xmax - 0.5), lim);
    int iy0 = (int)fmax(ceil(ymin - 0.5), -lim), iy1 = (int)fmin(floor(ymax - 0.5), lim);
    if (!V.wrap) {
        ix0 = ix0 > 0 ? ix0 : 0;
        iy0 = iy0 > 0 ? iy0 : 0;
        ix1 = ix1 < V.W - 1 ? ix1 : V.W - 1;
        iy1 = iy1 < V.H - 1 ? iy1 : V.H - 1;
    }
    if (ix0 > ix1 || iy0 > iy1) {
        count_tet(L, det6, flagged, cnt);
        return 0;
    }
    double qx[4], qy[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        qx[m] = PX[vi[m]] - (double)ix0;
        qy[m] = PY[vi[m]] - (double)iy0;
    }
    const double rho_m = 6.0 / fabs(det6);
    const double qscale = V.qpow == 1 ? 1.0 : (V.qpow == 0 ? 1.0 / (L.tet_mass * rho_m) : L.tet_mass * rho_m);
    const double mass_px = V.mass_px * qscale;
    double D[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const int b = kFace[a][0], c = kFace[a][1], d = kFace[a][2];
        const double ex = qx[c] - qx[b], ey = qy[c] - qy[b];
        const double fx = qx[d] - qx[b], fy = qy[d] - qy[b];
        D[a] = ex * fy - ey * fx;
    }
    if (D[0] == 0.0 || D[1] == 0.0 || D[2] == 0.0 || D[3] == 0.0) return -1;
    double b[6];
    uint32_t smask = 0u;
    double bmax = 0.0;
#pragma unroll
    for (int g = 0; g < 6; ++g) {
        const EdgeInfo E = kEdge[g];
        const double ck = (double)E.sk * D[E.l];
        const double cl = (double)E.sl * D[E.k];
        const double K = mass_px / (ck * fabs(cl));
        b[g] = -K * (qy[E.j] - qy[E.i]);
        if ((ck > 0 && cl > 0) || (ck < 0 && cl < 0)) {
            smask |= 1u << g;
            bmax = fmax(bmax, fabs(b[g]));
        }
    }
    // a triangle: the three edges avoiding one vertex; a quadrilateral: all
    // but a pair of opposite edges (local edges g and 5 - g are opposite)
    const bool tri = smask == 0x38u || smask == 0x26u || smask == 0x15u || smask == 0x0bu;
    const bool quad = smask == 0x1eu || smask == 0x2du || smask == 0x33u;
    if (!(tri || quad)) return -1;
    if (!(bmax <= crease_bmax)) {
        // steep along x: the line form, whatever the edge form's tests say;
        // its record holds the silhouette edges' face functions in edge
        // order (footprint's G functions a + b u + c v: K times the cross
        // product with the edge)
        RecHead R;
        R.bx = pack_range(ix0, ix1);
        R.by = pack_range(iy0, iy1);
        R.flags = (tri ? 3u : 4u) | REC_VALID;
        R.spare = 0u;
        // the payload is written where own_sink places it, a value at a time
        // (no place: the general setup takes the tetrahedron)
        Payload *const P = own_sink(t, R);
        if (!P) return -1;
        {
            int k = 0;
#pragma unroll
            for (int g = 0; g < 6; ++g) {
                if (!((smask >> g) & 1u)) continue;
                const EdgeInfo E = kEdge[g];
                const double dx = qx[E.j] - qx[E.i], dy = qy[E.j] - qy[E.i];
                const double ck = (double)E.sk * D[E.l];
                const double cl = (double)E.sl * D[E.k];
                const double K = mass_px / (ck * fabs(cl));
                P->c[3 * k + 0] = K * (dy * qx[E.i] - dx * qy[E.i]);
                P->c[3 * k + 1] = -K * dy;
                P->c[3 * k + 2] = K * dx;
                ++k;
            }
            for (int g = 3 * k; g < 14; ++g) P->c[g] = 0.0;
            P->h = R;
        }
        count_tet(L, det6, flagged, cnt);
        return 8;
    }
    // the period and margin tests of the edge form (as in setup_cube)
    if (!same_frame) return -1;
    uint32_t shift = 0x555u;
    if (V.wrap) {
        if (!(xmax - xmin < (double)V.W - 2.0)) return -1;
        const int pt = (int)floor(xmin * V.inv_W);
        shift = 0u;
        bool ok = true;
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            const EdgeSlot S = kEdgeSlots.s[t][q];
            const int m = S.ox + 2 * S.oy + 4 * S.oz;
            const int per = (int)((qpack >> (4 * m)) & 15u) - 2 - pt;
            ok = ok && per >= -1 && per <= 1;
            shift |= (uint32_t)(per + 1) << (2 * q);
        }
        if (!ok) return -1;
    } else if (!(xmin >= 1.0 && xmax <= (double)V.W - 1.0)) {
        return -1;
    }
    if (quad) {
        // the two diagonals (the edges off the silhouette) must cross
        const int g = smask == 0x1eu ? 0 : (smask == 0x2du ? 1 : 2);
        const EdgeInfo E = kEdge[0];
        const EdgeInfo F = kEdge[1];
        const EdgeInfo G = kEdge[2];
        const int i = g == 0 ? E.i : (g == 1 ? F.i : G.i), j = g == 0 ? E.j : (g == 1 ? F.j : G.j);
        const int k = g == 0 ? E.k : (g == 1 ? F.k : G.k), l = g == 0 ? E.l : (g == 1 ? F.l : G.l);
        auto px = [&](int v) { return v == 0 ? qx[0] : v == 1 ? qx[1] : v == 2 ? qx[2] : qx[3]; };
        auto py = [&](int v) { return v == 0 ? qy[0] : v == 1 ? qy[1] : v == 2 ? qy[2] : qy[3]; };
        const double den = (px(j) - px(i)) * (py(l) - py(k)) - (py(j) - py(i)) * (px(l) - px(k));
        if (den == 0.0) return -1;
    }
    count_tet(L, det6, flagged, cnt);
    uint32_t bits = 0u;
#pragma unroll
    for (int g = 0; g < 6; ++g) {
        const EdgeInfo E = kEdge[g];
        if (smask & (1u << g)) {
            kd[g] = fabs(b[g]);
            bits |= (b[g] > 0.0 ? 1u : 2u) << (2 * g);
        } else {
            // the ends' terms: edges (i, k), (i, l) and (j, k), (j, l)
            const int ik = local_edge(E.i, E.k), il = local_edge(E.i, E.l);
            const int jk = local_edge(E.j, E.k), jl = local_edge(E.j, E.l);
            const bool oi = (smask >> ik & 1u) && (smask >> il & 1u);
            const bool oj = (smask >> jk & 1u) && (smask >> jl & 1u);
            const double ti = fabs(b[ik] - b[il]), tj = fabs(b[jk] - b[jl]);
            kd[g] = oi && oj ? -0.5 * (ti + tj) : -(oi ? ti : tj);
        }
    }
    sil = bits;
    shf = shift;
    return tri ? 3 : 4;
}

// Setup of the six tetrahedra of lattice cube `cube` (EDGES: the edge form's
// code, used when V.edges is set; PASS 1 of it takes only the common cases,
// edge_tet_fast, and returns the tetrahedra left over in *todo_io, bit t for
// tetrahedron t, which PASS 2 then sets up by the general code; PASS 0 does
// both): gather and unwrap the
// corners, volume determinant with its FP64 fallback, footprint.  Each
// tetrahedron t's record goes to emit(t, head, payload) (flags 0 when it can
// cover no pixel centre; REC_EDGED when its creases went to its edges' slots,
// which setup_cube writes itself).
//
// The edge form's common path writes a line-form record (edge_tet_fast) to
// where own_sink(t, head) says, then calls own_done(t); without them the
// record is built in a local payload and goes to emit like the others.
template <int FORM, bool EDGES, int PASS, typename Emit, typename OwnSink, typename OwnDone>
TESS_HD inline void setup_cube(const LatticeParams &L, const ViewParams &V, int64_t cube, Emit &&emit,
                               CubeCounts &cnt, uint32_t *todo_io, OwnSink &&own_sink, OwnDone &&own_done);
template <int FORM, bool EDGES = false, int PASS = 0, typename Emit>
TESS_HD inline void setup_cube(const LatticeParams &L, const ViewParams &V, int64_t cube, Emit &&emit,
                               CubeCounts &cnt, uint32_t *todo_io = nullptr) {
    Payload own;
    setup_cube<FORM, EDGES, PASS>(
        L, V, cube, emit, cnt, todo_io, [&](int, const RecHead &) -> Payload * { return &own; },
        [&](int t) { emit(t, own.h, own); });
}
template <int FORM, bool EDGES, int PASS, typename Emit, typename OwnSink, typename OwnDone>
TESS_HD inline void setup_cube(const LatticeParams &L, const ViewParams &V, int64_t cube, Emit &&emit,
                               CubeCounts &cnt, uint32_t *todo_io, OwnSink &&own_sink, OwnDone &&own_done) {
    double X0[3], e[8][3];
    const bool moved = cube_corners(L, cube, X0, e);
    int64_t ci, cj, ck;
    cube_ijk(L, cube, ci, cj, ck);
    const int64_t nvert = (int64_t)L.d[0] * L.d[1] * L.d[2];
    // edge form: the cube's edges are placed from their own vertices (corners
    // of this cube).  That gives the same segments as this cube's corners if
    // the corners lie within half a box of each other along every axis (then
    // every vertex sees the others unmoved); without wrap the positions agree
    // only if, besides, no corner was moved by a box length (with wrap they
    // agree modulo the period)
    bool same_frame = V.wrap || !moved;
    if constexpr (EDGES) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            double lo = 0.0, hi = 0.0;
#pragma unroll
            for (int n = 1; n < 8; ++n) {
                lo = fmin(lo, e[n][a]);
                hi = fmax(hi, e[n][a]);
            }
            same_frame = same_frame && hi - lo < 0.5 * L.box[a];
        }
    }
    // x slope beyond which a footprint keeps the line form, from the image's
    // scale: the mass in view, or the measured integral of q
    const double crease_bmax = V.qsum ? *V.qsum * V.bmax_per_q : V.crease_bmax;
    // projected corners in pixel units
    const double b0[3] = {X0[0] - V.center[0], X0[1] - V.center[1], X0[2] - V.center[2]};
    const double Tc = V.rot[6] * b0[0] + V.rot[7] * b0[1] + V.rot[8] * b0[2];  // depth of corner 0
    double PX0 = (V.rot[0] * b0[0] + V.rot[1] * b0[1] + V.rot[2] * b0[2] - V.u_left) * V.inv_du;
    double PY0 = (V.rot[3] * b0[0] + V.rot[4] * b0[1] + V.rot[5] * b0[2] - V.v_bottom) * V.inv_dv;
    if (V.wrap) {  // a periodic image: move corner 0 into the first period
        PX0 -= (double)V.W * floor(PX0 * V.inv_W);
        PY0 -= (double)V.H * floor(PY0 * V.inv_H);
    }
    double PX[8], PY[8];
#pragma unroll
    for (int n = 0; n < 8; ++n) {
        PX[n] = PX0 + (V.rot[0] * e[n][0] + V.rot[1] * e[n][1] + V.rot[2] * e[n][2]) * V.inv_du;
        PY[n] = PY0 + (V.rot[3] * e[n][0] + V.rot[4] * e[n][1] + V.rot[5] * e[n][2]) * V.inv_dv;
    }
    // edge form under wrap: corner n's x in its own frame, where the edge
    // records it owns are placed, lies a whole number q_n of periods before
    // its x in this cube's frame
    // number of periods q_n, packed as q_n + 2 in 4 bits per corner
    uint32_t qpack = 0x22222222u;
    if constexpr (FORM == kFormPyramid && EDGES) {
        if (V.edges && V.wrap) {
            qpack = 0u;
#pragma unroll
            for (int n = 0; n < 8; ++n) {
                int64_t ii = ci + (n & 1), jj = cj + ((n >> 1) & 1), kk = ck + ((n >> 2) & 1);
                if (ii == L.d[0]) ii = 0;
                if (jj == L.d[1]) jj = 0;
                if (kk == L.d[2]) kk = 0;
                const double pe = vertex_px(L, V, ii + (int64_t)L.d[0] * (jj + (int64_t)L.d[1] * kk));
                const double q = fmin(fmax(rint((PX[n] - pe) * V.inv_W), -2.0), 13.0);
                qpack |= (uint32_t)((int)q + 2) << (4 * n);
            }
        }
    }
    // edge form: slot u of vertex w at u * nvert + w; the cube's corner n is
    // vertex cvert[n]
    int64_t cvert[8];
#pragma unroll
    for (int n = 0; n < 8; ++n) {
        const int64_t vx = ci + (n & 1) == L.d[0] ? 0 : ci + (n & 1);
        const int64_t vy = cj + ((n >> 1) & 1) == L.d[1] ? 0 : cj + ((n >> 1) & 1);
        const int64_t vz = ck + ((n >> 2) & 1) == L.d[2] ? 0 : ck + ((n >> 2) & 1);
        cvert[n] = vx + (int64_t)L.d[0] * (vy + (int64_t)L.d[1] * vz);
    }
    // every slot of the cube's tetrahedra is written (zeros for the
    // tetrahedra that keep their own record)
    auto edge_slots = [&](int t, const double kd[6], uint32_t sil, uint32_t shf) {
#pragma unroll
        for (int g = 0; g < 6; ++g) {
            const EdgeSlot S = kEdgeSlots.s[t][g];
            const int64_t slot = (int64_t)S.u * nvert + cvert[S.ox + 2 * S.oy + 4 * S.oz];
            V.kinks[slot] = kd[g];
            V.sil[slot] = (uint8_t)(((sil >> (2 * g)) & 3u) | (((shf >> (2 * g)) & 3u) << 2));
        }
    };
    // the tetrahedra the general code below takes
    uint32_t todo = 0x3fu;
    if constexpr (FORM == kFormPyramid && EDGES && PASS == 2) {
        todo = *todo_io;
    } else if constexpr (FORM == kFormPyramid && EDGES) {
        // edge form (this instantiation runs only with V.edges set): the
        // common case of each tetrahedron first, unrolled so that every
        // corner index is a constant
        todo = 0u;
#pragma unroll
        for (int t = 0; t < 6; ++t) {
            double kd[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
            uint32_t ksil = 0u, kshf = 0x555u;
            const int fast =
                edge_tet_fast(L, V, t, e, PX, PY, crease_bmax, same_frame, qpack, kd, ksil, kshf, own_sink, cnt);
            if (fast < 0) {
                todo |= 1u << t;
                continue;
            }
            if (fast == 8) {  // its own record is written
                own_done(t);
                edge_slots(t, kd, 0u, 0x555u);
                continue;
            }
            // (no payload: the head says whether its creases went to the edges)
            RecHead R;
            R.bx = 0;
            R.by = 0;
            R.flags = fast > 0 ? REC_EDGED | ((uint32_t)fast & REC_NG_MASK) : 0u;
            R.spare = fast > 0 ? ksil | (kshf << 12) : 0u;
            Payload P;
            P.h = R;
#pragma unroll
            for (int g = 0; g < 14; ++g) P.c[g] = 0.0;
            emit(t, R, P);
            edge_slots(t, kd, ksil, kshf);
        }
        if constexpr (PASS == 1) {
            *todo_io = todo;
            return;
        }
        if (todo == 0u) return;
    }
    // The general code, one copy of the body for the six tetrahedra (unrolled,
    // the setup kernels' code outgrew the instruction cache).
    auto general = [&](const double (&e)[8][3], const double (&PX)[8], const double (&PY)[8]) {
#pragma unroll 1
    for (int t = 0; t < 6; ++t) {
        if (!((todo >> t) & 1u)) continue;
        double kd[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};  // edge form: slope change per local edge
        double ev[4][3], pxv[4], pyv[4];                 // the tetrahedron's corners
        tet_corners(t, e, PX, PY, ev, pxv, pyv);
        // the record is built in registers and stored once, in whole lines
        RecHead R;
        R.bx = 0;
        R.by = 0;
        R.flags = 0;
        R.spare = 0;
        double pc[14];
#pragma unroll
        for (int g = 0; g < 14; ++g) pc[g] = 0.0;
        [&] {
            bool flagged;
            const double det6 = tet_det6(L, ev, flagged);
            count_tet(L, det6, flagged, cnt);
            if (det6 == 0.0) return;
            if constexpr (FORM == kFormSplat) {
                // the centroid method: a kernel of size h = |V|^(1/3) at the
                // projected centroid, carrying q |V|
                const double vol = fabs(det6) / 6.0;
                const double hh = cbrt(vol);
                const double rho = L.tet_mass * 6.0 / fabs(det6);
                const double qv = V.qpow == 0 ? 1.0 : (V.qpow == 1 ? rho : rho * rho);
                double cxp = 0.0, cyp = 0.0;
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    cxp += 0.25 * pxv[m];
                    cyp += 0.25 * pyv[m];
                }
                const double rx = 2.0 * hh * V.inv_du, ry = 2.0 * hh * V.inv_dv, lim = 1.0e8;
                int sx0 = (int)fmax(ceil(cxp - rx - 0.5), -lim), sx1 = (int)fmin(floor(cxp + rx - 0.5), lim);
                int sy0 = (int)fmax(ceil(cyp - ry - 0.5), -lim), sy1 = (int)fmin(floor(cyp + ry - 0.5), lim);
                if (!V.wrap) {
                    sx0 = sx0 > 0 ? sx0 : 0;
                    sy0 = sy0 > 0 ? sy0 : 0;
                    sx1 = sx1 < V.W - 1 ? sx1 : V.W - 1;
                    sy1 = sy1 < V.H - 1 ? sy1 : V.H - 1;
                }
                if (sx0 > sx1 || sy0 > sy1) return;
                pc[0] = cxp - (double)sx0;
                pc[1] = cyp - (double)sy0;
                pc[2] = 1.0 / (hh * V.inv_du);
                pc[3] = 1.0 / (hh * V.inv_dv);
                pc[4] = qv * vol * (10.0 / (7.0 * kPi * hh * hh));
                R.bx = pack_range(sx0, sx1);
                R.by = pack_range(sy0, sy1);
                R.flags = REC_SPLAT | REC_VALID;
                return;
            }
            if constexpr (FORM == kFormPersp) {
                // a camera at V.center: the vertices in the camera frame (the
                // raster clips each pixel's half-line against the faces), q,
                // and the pixel box of their projection onto the window
                const double rho = L.tet_mass * 6.0 / fabs(det6);
                const double qv = V.qpow == 0 ? 1.0 : (V.qpow == 1 ? rho : rho * rho);
                double ybase[3];
#pragma unroll
                for (int r = 0; r < 3; ++r) ybase[r] = V.rot[3 * r] * b0[0] + V.rot[3 * r + 1] * b0[1] + V.rot[3 * r + 2] * b0[2];
                if (V.splat || V.hybrid) {
                    // the centroid in the camera frame: a billboard (the centroid
                    // method, or beyond the hybrid's sphere around the camera)
                    double yc[3];
#pragma unroll
                    for (int r = 0; r < 3; ++r) {
                        double acc = 0.0;
#pragma unroll
                        for (int m = 0; m < 4; ++m)
                            acc += 0.25 * (ybase[r] + (V.rot[3 * r] * ev[m][0] + V.rot[3 * r + 1] * ev[m][1] +
                                                       V.rot[3 * r + 2] * ev[m][2]));
                        yc[r] = acc;
                    }
                    if (V.splat || sqrt(yc[0] * yc[0] + yc[1] * yc[1] + yc[2] * yc[2]) > V.lod_radius) {
                        if (!(yc[2] > 0.0)) return;  // behind the camera: not drawn
                        const double vol = fabs(det6) / 6.0;
                        const double hh = cbrt(vol), R2 = 2.0 * hh;
                        int ix0 = 0, ix1 = V.W - 1, iy0 = 0, iy1 = V.H - 1;
                        if (R2 < yc[2]) {  // the support disc's square on the billboard plane, a pixel of margin
                            const double lim = 1.0e8;
                            ix0 = max(ix0, (int)fmax(ceil(((yc[0] - R2) / yc[2] - V.u_left) * V.inv_du - 0.5) - 1.0, -lim));
                            ix1 = min(ix1, (int)fmin(floor(((yc[0] + R2) / yc[2] - V.u_left) * V.inv_du - 0.5) + 1.0, lim));
                            iy0 = max(iy0, (int)fmax(ceil(((yc[1] - R2) / yc[2] - V.v_bottom) * V.inv_dv - 0.5) - 1.0, -lim));
                            iy1 = min(iy1, (int)fmin(floor(((yc[1] + R2) / yc[2] - V.v_bottom) * V.inv_dv - 0.5) + 1.0, lim));
                        }
                        if (ix0 > ix1 || iy0 > iy1) return;
                        pc[0] = yc[0] / yc[2];
                        pc[1] = yc[1] / yc[2];
                        pc[2] = yc[2];
                        pc[3] = 1.0 / hh;
                        pc[4] = qv * vol * (10.0 / (7.0 * kPi * hh * hh));
                        R.bx = pack_range(ix0, ix1);
                        R.by = pack_range(iy0, iy1);
                        R.flags = REC_SPLAT | REC_VALID;
                        return;
                    }
                }
                bool behind = false;
                double umin = 1e300, umax = -1e300, vmin = 1e300, vmax = -1e300;
                // frustum culling: the window's edges widened by a pixel; a
                // tetrahedron with all four vertices beyond one side plane
                // (u z < ul, u z > ur, ...) or at or behind the camera is unseen
                const double ul = V.u_left - 1.0 / V.inv_du, ur = -V.u_left + 1.0 / V.inv_du;
                const double vb = V.v_bottom - 1.0 / V.inv_dv, vt = -V.v_bottom + 1.0 / V.inv_dv;
                int out_l = 0, out_r = 0, out_b = 0, out_t = 0, out_z = 0;
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    double yv[3];
#pragma unroll
                    for (int r = 0; r < 3; ++r)
                        yv[r] = ybase[r] + (V.rot[3 * r] * ev[m][0] + V.rot[3 * r + 1] * ev[m][1] +
                                            V.rot[3 * r + 2] * ev[m][2]);
                    pc[3 * m + 0] = yv[0];
                    pc[3 * m + 1] = yv[1];
                    pc[3 * m + 2] = yv[2];
                    if (!(yv[2] > 0.0)) behind = true;
                    out_z += yv[2] > 0.0 ? 0 : 1;
                    out_l += yv[0] < ul * yv[2] ? 1 : 0;
                    out_r += yv[0] > ur * yv[2] ? 1 : 0;
                    out_b += yv[1] < vb * yv[2] ? 1 : 0;
                    out_t += yv[1] > vt * yv[2] ? 1 : 0;
                    const double pu = yv[0] / yv[2], pv = yv[1] / yv[2];
                    umin = fmin(umin, pu); umax = fmax(umax, pu);
                    vmin = fmin(vmin, pv); vmax = fmax(vmax, pv);
                }
                pc[12] = qv;
                if (out_z == 4 || out_l == 4 || out_r == 4 || out_b == 4 || out_t == 4) {
#pragma unroll
                    for (int g = 0; g < 14; ++g) pc[g] = 0.0;
                    return;
                }
                int ix0 = 0, ix1 = V.W - 1, iy0 = 0, iy1 = V.H - 1;  // behind: any pixel
                if (!behind) {  // pixel centres in the projected box, one pixel of margin
                    const double lim = 1.0e8;
                    ix0 = max(ix0, (int)fmax(ceil((umin - V.u_left) * V.inv_du - 0.5) - 1.0, -lim));
                    ix1 = min(ix1, (int)fmin(floor((umax - V.u_left) * V.inv_du - 0.5) + 1.0, lim));
                    iy0 = max(iy0, (int)fmax(ceil((vmin - V.v_bottom) * V.inv_dv - 0.5) - 1.0, -lim));
                    iy1 = min(iy1, (int)fmin(floor((vmax - V.v_bottom) * V.inv_dv - 0.5) + 1.0, lim));
                }
                if (ix0 > ix1 || iy0 > iy1) {
#pragma unroll
                    for (int g = 0; g < 14; ++g) pc[g] = 0.0;
                    return;
                }
                R.bx = pack_range(ix0, ix1);
                R.by = pack_range(iy0, iy1);
                R.flags = REC_PERSP | REC_VALID;
                return;
            }
            // ---- screen footprint (FP64)
            double xmin = pxv[0], xmax = pxv[0], ymin = pyv[0], ymax = pyv[0];
#pragma unroll
            for (int m = 1; m < 4; ++m) {
                xmin = fmin(xmin, pxv[m]); xmax = fmax(xmax, pxv[m]);
                ymin = fmin(ymin, pyv[m]); ymax = fmax(ymax, pyv[m]);
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
            if (ix0 > ix1 || iy0 > iy1) return;
            double qx[4], qy[4];
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                qx[m] = pxv[m] - (double)ix0;
                qy[m] = pyv[m] - (double)iy0;
            }
            const double rho_m = 6.0 / fabs(det6);  // rho / m
            if constexpr (FORM == kFormFace) {
                // depth slab: the face form, q times the clipped chord
                double T[4];
#pragma unroll
                for (int m = 0; m < 4; ++m)
                    T[m] = Tc + V.rot[6] * ev[m][0] + V.rot[7] * ev[m][1] + V.rot[8] * ev[m][2];
                const double rho = L.tet_mass * rho_m;
                const double qv = V.qpow == 0 ? 1.0 : (V.qpow == 1 ? rho : rho * rho);
                uint32_t ff = 0;
                if (!face_payload(qx, qy, T, V.slab_t[0], V.slab_t[1], qv, pc, ff)) {
#pragma unroll
                    for (int g = 0; g < 14; ++g) pc[g] = 0.0;
                    return;
                }
                R.bx = pack_range(ix0, ix1);
                R.by = pack_range(iy0, iy1);
                R.flags = ff | REC_FACE | REC_VALID;
                return;
            }
            // q dl = (q / rho) rho dl: the density footprint with its mass scaled
            // by rho^(qpow - 1), rho = 6 m / |6V|
            const double qscale = V.qpow == 1 ? 1.0 : (V.qpow == 0 ? 1.0 / (L.tet_mass * rho_m) : L.tet_mass * rho_m);
            Footprint fp;
            if (!footprint(qx, qy, V.mass_px * qscale, fp)) return;
            R.bx = pack_range(ix0, ix1);
            R.by = pack_range(iy0, iy1);
            R.flags = (uint32_t)fp.ng | ((uint32_t)fp.nw << REC_NW_SHIFT) | fp.ties | REC_VALID;
            // crease form unless the footprint is steep along x: its kinks' rounding
            // would then carry along the row sums (steep slivers keep the line form,
            // whose rows without a pixel centre are skipped)
            double bmax = 0.0;
#pragma unroll
            for (int g = 0; g < 4; ++g) bmax = fmax(bmax, fabs(fp.c[3 * g + 1]));
            const bool crease = fp.nw == 0 && bmax <= crease_bmax;
            if constexpr (FORM == kFormPyramid && EDGES) {
                // edge form: a tetrahedron within the image's columns (a
                // pixel of margin; under wrap, within one period) hands its
                // creases to the mesh edges, where they are summed over the
                // tetrahedra around each edge (when same_frame holds)
                // Without wrap the tetrahedron must lie within the image's
                // columns (a pixel of margin).  With wrap any one narrower
                // than the image will do: in the frame that puts its left
                // end in the first period, an edge lies s periods from
                // where its own vertex places it (s in -1..1, kept in bits
                // 2-3 of the silhouette kind as s + 1), and the raster
                // corrects the rows at the period's seam from it.
                uint32_t sil = 0u;
                bool take = crease && V.edges && same_frame;
                uint32_t shift = 0x555u;  // s + 1 = 1 for all six edges
                if (take && V.wrap) {
                    const int pt = (int)floor(xmin * V.inv_W);  // this frame's period of xmin
                    take = xmax - xmin < (double)V.W - 2.0;
                    shift = 0u;
#pragma unroll
                    for (int q = 0; q < 6; ++q) {
                        const EdgeSlot S = kEdgeSlots.s[t][q];
                        const int m = S.ox + 2 * S.oy + 4 * S.oz;
                        const int per = (int)((qpack >> (4 * m)) & 15u) - 2 - pt;
                        take = take && per >= -1 && per <= 1;
                        shift |= (uint32_t)(per + 1) << (2 * q);
                    }
                } else if (take) {
                    take = xmin >= 1.0 && xmax <= (double)V.W - 1.0;
                }
                if (take && crease_kinks(qx, qy, fp, kd, sil)) {
                    R.flags = REC_EDGED | (uint32_t)fp.ng;
                    R.spare = sil | (shift << 12);
                    return;
                }
            }
            if (crease && crease_payload(qx, qy, fp, pc)) {
                R.flags |= REC_CREASE;
                R.spare = crease_profile(pc, iy1 - iy0 + 1);
            } else {
#pragma unroll
                for (int g = 0; g < 12; ++g) pc[g] = fp.c[g];
            }
        }();
        Payload P;
        P.h = R;
#pragma unroll
        for (int g = 0; g < 14; ++g) P.c[g] = pc[g];
        emit(t, R, P);
        if constexpr (FORM == kFormPyramid && EDGES) {
            const bool edged = (R.flags & REC_EDGED) != 0u;
            edge_slots(t, kd, edged ? R.spare & 0xfffu : 0u, edged ? R.spare >> 12 : 0x555u);
        }
    }
    };
    general(e, PX, PY);
}

// Pixel box of an edge from (ax, ay) to (bx, by): the columns that receive
// its deposits, floor(x - 1/2) + 1 (+ kRightReach), and the rows whose centre
// lies in [min y, max y), clipped to the image without wrap.  False when it
// has no row there.  The edge records and the raster both take it from here.
TESS_HD inline bool edge_box(double ax, double ay, double bx, double by, const BinParams &B, int &ix0, int &ix1,
                             int &iy0, int &iy1) {
    const double lim = 1.0e8;
    const double xlo = fmin(ax, bx), xhi = fmax(ax, bx), ylo = fmin(ay, by), yhi = fmax(ay, by);
    ix0 = (int)fmax(floor(xlo - 0.5), -lim) + 1;
    ix1 = (int)fmin(floor(xhi - 0.5), lim);
    iy0 = (int)fmax(ceil(ylo - 0.5), -lim);
    iy1 = (int)fmin(ceil(yhi - 0.5), lim) - 1;
    if (ix1 < ix0) ix1 = ix0;
    if (!B.wrap) {
        ix0 = ix0 > 0 ? ix0 : 0;
        iy0 = iy0 > 0 ? iy0 : 0;
        ix1 = ix1 < B.W - 1 ? ix1 : B.W - 1;
        iy1 = iy1 < B.H - 1 ? iy1 : B.H - 1;
    }
    return ix0 <= ix1 && iy0 <= iy1;
}

// Edge records of lattice vertex v (edge form), at head[tau * nvert] and
// ecoef[tau * nvert] for its edge kinds tau (the records are stored kind by
// kind, so that neighbouring vertices write neighbouring records): for each of its seven edges
// the sum of the slope changes setup wrote for the tetrahedra around it that
// handed their creases to their edges, the counts of those for which it is
// an entering or leaving silhouette edge, and its projected endpoints in the
// frame of the cube with corner 0 at v (the frame setup uses for that cube).
// An edge with nothing to draw gets flags 0.
TESS_HD inline void setup_vertex_edges(const LatticeParams &L, const ViewParams &V, int64_t v,
                                       RecHead *head, EdgePayload *ecoef) {
    const int64_t nvert = (int64_t)L.d[0] * L.d[1] * L.d[2];
    const int64_t rest = v / L.d[0];
    const int64_t i = v - rest * L.d[0];
    const int64_t k = rest / L.d[1];
    const int64_t j = rest - k * L.d[1];
    // corners 0..4 of the cube at v (they may lie past a non-periodic lattice)
    double X0[3] = {0.0, 0.0, 0.0}, e[5][3];
    bool has[5];
#pragma unroll
    for (int n = 0; n < 5; ++n) {
        int64_t ii = i + (n & 1), jj = j + ((n >> 1) & 1), kk = k + ((n >> 2) & 1);
        if (L.periodic) {
            if (ii == L.d[0]) ii = 0;
            if (jj == L.d[1]) jj = 0;
            if (kk == L.d[2]) kk = 0;
        }
        has[n] = ii < L.d[0] && jj < L.d[1] && kk < L.d[2];
        e[n][0] = e[n][1] = e[n][2] = 0.0;
        if (!has[n]) continue;
        const int64_t id = ii + (int64_t)L.d[0] * (jj + (int64_t)L.d[1] * kk);
        const double p[3] = {(double)L.x[id], (double)L.y[id], (double)L.z[id]};
        if (n == 0) {
            X0[0] = p[0]; X0[1] = p[1]; X0[2] = p[2];
        } else {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                double d = p[a] - X0[a];
                if (L.periodic) d -= L.box[a] * ceil(d / L.box[a] - 0.5);
                e[n][a] = d;
            }
        }
    }
    const double b0[3] = {X0[0] - V.center[0], X0[1] - V.center[1], X0[2] - V.center[2]};
    const double PX0 = vertex_px(L, V, v);
    double PY0 = (V.rot[3] * b0[0] + V.rot[4] * b0[1] + V.rot[5] * b0[2] - V.v_bottom) * V.inv_dv;
    if (V.wrap) PY0 -= (double)V.H * floor(PY0 * V.inv_H);
    // the slope changes by period offset of the edges that have offsets: kept
    // until every slot of this vertex has been read, then written over slots
    // 7 g + tau of this vertex (the slots' edge-major view, BinParams::groups)
    double G[7][3];
    uint32_t offs = 0u;
#pragma unroll
    for (int tau = 0; tau < 7; ++tau) {
        RecHead R;
        R.bx = 0; R.by = 0; R.flags = 0; R.spare = 0;
        EdgePayload P;
        G[tau][0] = G[tau][1] = G[tau][2] = 0.0;
        [&] {
            const int ca = kEdgeEnds[tau][0], cb = kEdgeEnds[tau][1];
            if (!has[ca] || !has[cb]) return;
            double D[3] = {0.0, 0.0, 0.0};  // by period offset s + 1
            uint32_t cnt = 0u;               // 3 bits each: entering s = -1, 0, 1, then leaving
            for (int u = kEdgeFirst[tau]; u < kEdgeFirst[tau + 1]; ++u) {
                const EdgeUse U = kEdgeUse[u];
                if (!L.periodic) {  // slots of cubes past the lattice are never written
                    const int64_t ci = i + U.dx, cj = j + U.dy, ck = k + U.dz;
                    if (ci < 0 || cj < 0 || ck < 0 || ci >= L.c[0] || cj >= L.c[1] || ck >= L.c[2]) continue;
                }
                const double d = V.kinks[(int64_t)u * nvert + v];
                const uint32_t sb = V.sil[(int64_t)u * nvert + v];
                const uint32_t g = (sb >> 2) & 3u, kind = sb & 3u;
                D[0] += g == 0u ? d : 0.0;
                D[1] += g == 1u ? d : 0.0;
                D[2] += g == 2u ? d : 0.0;
                if (kind != 0u) cnt += 1u << (3 * g + (kind == 2u ? 9 : 0));
            }
            if (D[0] == 0.0 && D[1] == 0.0 && D[2] == 0.0 && cnt == 0u) return;
            double ax = PX0, ay = PY0, bx = PX0, by = PY0;
#pragma unroll
            for (int n = 1; n < 5; ++n) {
                const double px = PX0 + (V.rot[0] * e[n][0] + V.rot[1] * e[n][1] + V.rot[2] * e[n][2]) * V.inv_du;
                const double py = PY0 + (V.rot[3] * e[n][0] + V.rot[4] * e[n][1] + V.rot[5] * e[n][2]) * V.inv_dv;
                if (n == ca) { ax = px; ay = py; }
                if (n == cb) { bx = px; by = py; }
            }
            BinParams Bv{};
            Bv.W = V.W;
            Bv.H = V.H;
            Bv.wrap = V.wrap;
            int ix0, ix1, iy0, iy1;
            // (a row's centre strictly inside the y range: the edge is not
            // horizontal, so sl below is finite)
            if (!edge_box(ax, ay, bx, by, Bv, ix0, ix1, iy0, iy1)) return;
            // the endpoints in the record frame (exact: integer offsets)
            const double Px = ax - (double)ix0, Py = ay - (double)iy0;
            const double Qx = bx - (double)ix0, Qy = by - (double)iy0;
            P.sl = (Qx - Px) / (Qy - Py);
            P.base = fma(0.5 - Py, P.sl, Px - 0.5);
            P.D = D[0] + D[1] + D[2];
            const bool off = D[0] != 0.0 || D[2] != 0.0;
            const uint32_t offbits = (D[0] != 0.0 ? kEdgeMinus : 0u) | (D[2] != 0.0 ? kEdgePlus : 0u);
            R.bx = pack_range(ix0, ix1);
            R.by = pack_range(iy0, iy1);
            R.flags = REC_EDGE | REC_VALID;
            R.spare = cnt;
            // (an edge narrower than the image, as those of the tetrahedra
            // that hand their creases to their edges are: the width fits)
            P.bx = ((uint32_t)(uint16_t)(int16_t)ix0) | ((uint32_t)(ix1 - ix0) << 16) | offbits;
            P.by = R.by;
            if (off) {
                G[tau][0] = D[0];
                G[tau][1] = D[1];
                G[tau][2] = D[2];
                offs |= 1u << tau;
            }
        }();
        head[tau * nvert] = R;
        // the whole 32 bytes (a partial write would cost a read-modify-write)
        if (R.flags & REC_VALID) ecoef[tau * nvert] = P;
    }
    if (offs) {
#pragma unroll
        for (int tau = 0; tau < 7; ++tau) {
            if (!(offs & (1u << tau))) continue;
#pragma unroll
            for (int g = 0; g < 3; ++g) V.kinks[(int64_t)(7 * g + tau) * nvert + v] = G[tau][g];
        }
    }
}

// ---------------------------------------------------------------- binning
// Tiles of one axis touched by the pixel range [b0, b1] (tile size T):
// `count` tiles starting at `start`, taken modulo the tile count under wrap.
TESS_HD inline void axis_tiles(int b0, int b1, int n, int T, int ntiles, int wrap,
                                  int &start, int &count) {
    if (!wrap) {
        const int lo = max(b0, 0), hi = min(b1, n - 1);
        if (lo > hi) { start = 0; count = 0; return; }
        start = floor_div(lo, T);
        count = floor_div(hi, T) - start + 1;
        return;
    }
    if (b1 - b0 + 1 >= n) { start = 0; count = ntiles; return; }
    const int a = imod(b0, n);
    const int b = a + (b1 - b0);
    if (b < n) { start = floor_div(a, T); count = floor_div(b, T) - start + 1; return; }
    const int ta = floor_div(a, T), tb = floor_div(b - n, T);
    if (tb >= ta) { start = 0; count = ntiles; return; }
    start = ta;
    count = ntiles - ta + tb + 1;
}

// Offsets k (in units of the image size) for which tile pixels [t0, t1]
// shifted by k*n meet [b0, b1]; a box inside the image needs only k = 0.
TESS_HD inline void axis_offsets(int t0, int t1, int b0, int b1, int n, int wrap, int &k0, int &k1) {
    if (!wrap || (b0 >= 0 && b1 < n)) {
        k0 = 0;
        k1 = 0;
        return;
    }
    k0 = ceil_div(b0 - t1, n);
    k1 = floor_div(b1 - t0, n);
}

// Columns a record writes: its pixel box plus two, since the last break point
// of a row (the end of the footprint) writes the two entries after it.
// Sorts eight keys into descending order (a 19-comparator network of depth 6).
TESS_HD inline void sort8_desc(uint32_t a[8]) {
    constexpr int kNet[19][2] = {{0, 2}, {1, 3}, {4, 6}, {5, 7}, {0, 4}, {1, 5}, {2, 6},
                                 {3, 7}, {0, 1}, {2, 3}, {4, 5}, {6, 7}, {2, 4}, {3, 5},
                                 {1, 4}, {3, 6}, {1, 2}, {3, 4}, {5, 6}};
#pragma unroll
    for (int i = 0; i < 19; ++i) {
        const uint32_t x = a[kNet[i][0]], y = a[kNet[i][1]];
        a[kNet[i][0]] = x > y ? x : y;
        a[kNet[i][1]] = x > y ? y : x;
    }
}

// Offset (pixels) that decides on which side of a crease a sample exactly on
// it falls: far above the rounding of a crossing (about 1e-13 px over a
// footprint). A crossing closer than this to a sample counts as on it, which
// moves the fragment count only (the deposits use the exact crossing).
constexpr double kSampleEps = 1e-10;
constexpr int kRightReach = 2;

// Candidate tiles of one record: tx = (sx + s % cx) mod ntx, ty = (sy + s / cx)
// mod nty for s < count = cx * cy.  Every tile of the box is a candidate:
// the tiles are wide row bands, so the box and the footprint meet nearly the
// same ones.
struct TileRange {
    int sx, cx, sy, cy, count;
};

TESS_HD inline TileRange tet_tiles(const RecHead &r, const BinParams &B) {
    TileRange t;
    axis_tiles(range_lo(r.bx), range_hi(r.bx) + kRightReach, B.W, B.Tw, B.ntx, B.wrap, t.sx, t.cx);
    axis_tiles(range_lo(r.by), range_hi(r.by), B.H, B.Th, B.nty, B.wrap, t.sy, t.cy);
    t.count = t.cx * t.cy;
    return t;
}

TESS_HD inline int tet_tile(const BinParams &B, const TileRange &t, int s) {
    int tx = t.sx + s % t.cx, ty = t.sy + s / t.cx;
    if (tx >= B.ntx) tx -= B.ntx;
    if (ty >= B.nty) ty -= B.nty;
    return ty * B.ntx + tx;
}

// Work class of a (record, tile) pair, 0 <= class < 32.  The raster's lanes
// step through their creases together, so a wavefront's time follows its
// longest lanes; pairs of one class have about the same number of active
// creases and rows, and the raster hands a wavefront's pairs to its lanes in
// class order.  Estimated from the head alone (the row profile of a
// crease-form record; every other record is class 0): the creases whose rows
// meet the tile's, and their mean row count in it in quarters of the tile
// height.  Only the order of work depends on it.
struct ClassRows {
    int lo[8], hi[8];  // record rows of each crease slot (empty: lo > hi)
    bool crease;
};

TESS_HD inline ClassRows class_rows(const RecHead &r) {
    ClassRows cr;
    cr.crease = (r.flags & REC_CREASE) != 0;
    const int sh = (int)((r.spare >> 25) & 31u);
    int yb[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) yb[v] = ((int)((r.spare >> (5 * v)) & 31u) << sh) + ((1 << sh) >> 1);
    const int m = (int)(r.flags & REC_NG_MASK);
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const int k = c & 3;
        const int k1 = k + 1 < m ? k + 1 : 0;
        const int P = c < 4 ? yb[k] : yb[4], Q = c < 4 ? yb[k1] : yb[k];
        cr.lo[c] = k < m ? min(P, Q) : 1;
        cr.hi[c] = k < m ? max(P, Q) - 1 : 0;
    }
    return cr;
}

// the class for the tile row ty, from class_rows of the record
TESS_HD inline int row_class(const ClassRows &cr, const RecHead &r, const BinParams &B, int ty) {
    if (!cr.crease) return 0;
    const int ty0 = ty * B.Th;
    const int rows = min(B.Th, B.H - ty0);
    int lo = ty0 - range_lo(r.by);  // the tile's first row in record rows (the period nearest)
    if (B.wrap) {
        if (lo < 0) lo += B.H;
        if (lo >= B.H) lo -= B.H;
    }
    const int hi = lo + rows - 1;
    int nact = 0, nrows = 0;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const int a = max(cr.lo[c], lo), b = min(cr.hi[c], hi);
        nact += a <= b ? 1 : 0;
        nrows += a <= b ? b - a + 1 : 0;
    }
    if (nact == 0) return 0;
    const int full = nact * rows;  // fill = floor(4 nrows / full), at most 3
    const int fill = 4 * nrows >= 3 * full ? 3 : 4 * nrows >= 2 * full ? 2 : 4 * nrows >= full ? 1 : 0;
    return (min(nact, 8) - 1) * 4 + fill;
}

TESS_HD inline int pair_class(const RecHead &r, const BinParams &B, int ty) {
    return row_class(class_rows(r), r, B, ty);
}

// ----------------------------------------------------------------- raster
// Along one pixel row the footprint f is piecewise linear in x: the lower
// envelope of the lines G_g(., Y), cut to where it is positive and to the
// walls.  Sampled at the pixel centres u = 0, 1, ..., n-1 of a tile row it is
// fully described by its second differences
//     A[k] = f(k) - 2 f(k-1) + f(k-2)      (f(-1) = f(-2) = 0),
// which vanish except next to the break points, and f is recovered by two
// running sums.  A break point at u* after which the function gains a step J
// and a slope change D (it adds J + D (k - u*) to every sample k > u*) adds
//     J + D phi  to A[j]  and  D (1 - phi) - J  to A[j+1],
// j = floor(u*) + 1, phi = j - u*.  The running sums run along whole image
// rows, so every break point keeps its true position and a tile writes only
// its own entries; break points left of the image are moved to its left edge
// (half a pixel before column 0) with J taken there, which gives the same
// samples in the image.

constexpr double kInf = __builtin_huge_val();

// Per-record geometry of the row spans, in the record frame.  The lines are
// sorted by decreasing x slope b, so that along a row the envelope visits them
// in index order; lines beyond ng are fillers (never active, bound nothing).
struct SpanGeom {
    double a[4], b[4], c[4];   // G_g = a + b X + c Y  (fillers: a = +inf)
    double r[4];               // -1 / b_g (G_g = 0 at X = r_g * (a_g + c_g Y))
    double q[6];               // pair p = (h < g): 1 / (b_h - b_g), 1 for fillers
    uint32_t lpos, lneg;       // bit g: b_g > 0 (left bound), b_g < 0 (right bound)
    uint32_t flat;             // bit g: b_g == 0 (G_g constant along a row)
    uint32_t fill;             // bit g: filler line
    uint32_t par;              // bit p: parallel pair (b_h == b_g)
    uint32_t nw, ties;         // walls: count and tie bits
    uint32_t wall0;            // index of the first wall coefficient (3 ng)
};

// Pair index of lines (h, g), h < g < 4.
constexpr int kPair[4][4] = {{-1, 0, 1, 2}, {0, -1, 3, 4}, {1, 3, -1, 5}, {2, 4, 5, -1}};

TESS_HD inline void cswap_line(double &a0, double &b0, double &c0, double &k0, double &a1, double &b1,
                               double &c1, double &k1) {
    const bool sw = k1 > k0;
    const double ta = sw ? a1 : a0, tb = sw ? b1 : b0, tc = sw ? c1 : c0, tk = sw ? k1 : k0;
    a1 = sw ? a0 : a1; b1 = sw ? b0 : b1; c1 = sw ? c0 : c1; k1 = sw ? k0 : k1;
    a0 = ta; b0 = tb; c0 = tc; k0 = tk;
}

TESS_HD inline void span_geom(uint32_t flags, const double *cf, SpanGeom &G) {
    const int ng = (int)(flags & REC_NG_MASK);
    double a[4], b[4], c[4], k[4];
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        const bool real = g < ng;
        a[g] = real ? cf[3 * g] : kInf;
        b[g] = real ? cf[3 * g + 1] : 0.0;
        c[g] = real ? cf[3 * g + 2] : 0.0;
        k[g] = real ? b[g] : -kInf;
    }
    // sorting network, decreasing key; fillers (key -inf) end last
    cswap_line(a[0], b[0], c[0], k[0], a[1], b[1], c[1], k[1]);
    cswap_line(a[2], b[2], c[2], k[2], a[3], b[3], c[3], k[3]);
    cswap_line(a[0], b[0], c[0], k[0], a[2], b[2], c[2], k[2]);
    cswap_line(a[1], b[1], c[1], k[1], a[3], b[3], c[3], k[3]);
    cswap_line(a[1], b[1], c[1], k[1], a[2], b[2], c[2], k[2]);
    G.lpos = G.lneg = G.flat = G.fill = G.par = 0;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        G.a[g] = a[g];
        G.b[g] = b[g];
        G.c[g] = c[g];
        const bool real = g < ng;
        G.r[g] = (real && b[g] != 0.0) ? -1.0 / b[g] : 0.0;
        if (!real) G.fill |= 1u << g;
        else if (b[g] > 0.0) G.lpos |= 1u << g;
        else if (b[g] < 0.0) G.lneg |= 1u << g;
        else G.flat |= 1u << g;
    }
#pragma unroll
    for (int h = 0; h < 4; ++h)
#pragma unroll
        for (int g = h + 1; g < 4; ++g) {
            const int p = kPair[h][g];
            const double den = b[h] - b[g];  // >= 0 by the sort
            double q = 1.0;
            if (g < ng) {
                if (den > 0.0) q = 1.0 / den;
                else G.par |= 1u << p;
            }
            G.q[p] = q;
        }
    G.nw = (flags >> REC_NW_SHIFT) & 3u;
    G.ties = (flags & REC_TIE0 ? 1u : 0u) | (flags & REC_TIE1 ? 2u : 0u);
    G.wall0 = 3u * (uint32_t)ng;
}

// One row of one record against one tile row, evaluated in the record frame
// (sample u = j at the record's column j, X = u + 1/2; row centre Y), so that
// every tile computes the same break points: the tile's samples are
// u = shift .. shift + n - 1, and the image row spans u in (ulo, uhi) (record
// frame).  cf: the record's coefficients (walls are read from there).  Break
// points sit at their true positions, except that pieces starting left of the
// image start at ulo; only the tile's own entries are written: dep(j, v) adds
// v to A[j] for the tile column 0 <= j < n.  Returns the number of the tile's
// samples with f > 0.
template <typename Dep>
TESS_HD inline uint32_t row_span(const SpanGeom &G, const double *cf, int shift, double Y, int n,
                                 double ulo, double uhi, Dep &&dep, uint32_t &kinks) {
    constexpr double X0 = 0.5;
    double A[4];
#pragma unroll
    for (int g = 0; g < 4; ++g) A[g] = G.a[g] + G.b[g] * X0 + G.c[g] * Y;  // G_g at sample u: A + b u
    double uL = ulo, uR = uhi;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        const double z = A[g] * G.r[g];  // zero of G_g along the row
        uL = fmax(uL, ((G.lpos >> g) & 1u) ? z : -kInf);
        uR = fmin(uR, ((G.lneg >> g) & 1u) ? z : kInf);
    }
    if (G.flat) {
#pragma unroll
        for (int g = 0; g < 4; ++g)
            if (((G.flat >> g) & 1u) && !(A[g] > 0.0)) return 0;
    }
    if (G.nw) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            if (q >= (int)G.nw) break;
            const double w0 = cf[G.wall0 + 3 * q], w1 = cf[G.wall0 + 3 * q + 1], w2 = cf[G.wall0 + 3 * q + 2];
            const bool tie = (G.ties >> q) & 1u;
            if (w1 == 0.0) {
                const double wv = w0 + w2 * Y;
                if (!(wv > 0.0 || (wv == 0.0 && tie))) return 0;
            } else {
                // admitted samples: W > 0 (or W == 0 with the tie bit)
                const double uw = -(w0 + w2 * Y) / w1 - X0;
                if (w1 > 0.0) uL = fmax(uL, (tie ? ceil(uw) : floor(uw) + 1.0) - 0.5);
                else uR = fmin(uR, (tie ? floor(uw) : ceil(uw) - 1.0) + 0.5);
            }
        }
    }
    if (!(ceil(uR) - floor(uL) > 1.0)) return 0;  // no sample in (uL, uR)
    // the tile's samples in (uL, uR)
    const double dshift = (double)shift;
    const double span = ceil(fmin(uR, dshift + (double)n - 0.5)) - floor(fmax(uL, dshift - 0.5)) - 1.0;
    double x[6];
#pragma unroll
    for (int h = 0; h < 4; ++h)
#pragma unroll
        for (int g = h + 1; g < 4; ++g) {
            const int p = kPair[h][g];
            x[p] = (A[g] - A[h]) * G.q[p];  // G_g < G_h right of x (+inf for a filler g)
        }
    if (G.par) {
#pragma unroll
        for (int h = 0; h < 4; ++h)
#pragma unroll
            for (int g = h + 1; g < 4; ++g) {
                const int p = kPair[h][g];
                if ((G.par >> p) & 1u) x[p] = A[h] - A[g] > 0.0 ? -kInf : kInf;
            }
    }
    double lo[4], hi[4];
    lo[0] = uL;
    hi[0] = fmin(fmin(uR, x[0]), fmin(x[1], x[2]));
    lo[1] = fmax(uL, x[0]);
    hi[1] = fmin(uR, fmin(x[3], x[4]));
    lo[2] = fmax(uL, fmax(x[1], x[3]));
    hi[2] = fmin(uR, x[5]);
    lo[3] = fmax(fmax(uL, x[2]), fmax(x[4], x[5]));
    hi[3] = uR;
    // the envelope's pieces that hold a sample, left to right; each start is
    // a break point relative to the previous piece
    bool have = false;
    double pA = 0.0, pB = 0.0, pHi = 0.0;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        if (!((G.fill >> g) & 1u) && floor(hi[g]) > floor(lo[g])) {  // an integer in (lo, hi]
            const double u = lo[g];
            const double J = (A[g] + G.b[g] * u) - (have ? pA + pB * u : 0.0);
            const double D = G.b[g] - (have ? pB : 0.0);
            const double fj = floor(u);
            const int j = (int)fj + 1 - shift;
            const double v1 = J + D * ((fj + 1.0) - u);
            if (j >= 0 && j < n) dep(j, v1);
            if (j >= -1 && j + 1 < n) dep(j + 1, D - v1);
            have = true;
            ++kinks;
            pA = A[g];
            pB = G.b[g];
            pHi = hi[g];
        }
    }
    if (have) {
        ++kinks;
        const double u = pHi;
        const double J = -(pA + pB * u), D = -pB;
        const double fj = floor(u);
        const int j = (int)fj + 1 - shift;
        const double v1 = J + D * ((fj + 1.0) - u);
        if (j >= 0 && j < n) dep(j, v1);
        if (j >= -1 && j + 1 < n) dep(j + 1, D - v1);
    }
    return span > 0.0 ? (uint32_t)span : 0u;
}

// All spans of one record in one tile (every periodic offset that meets it):
// tile pixels [tx0, tx0 + n) x [ty0, ty0 + rows).  dep(row, j, v) adds v to
// the tile's A[row][j].  Returns the covered sample count; spans counts the
// rows visited, kinks the break points placed.
template <typename Dep>
TESS_HD inline uint32_t raster_pair(const RecHead &h, const double *cf, const BinParams &B, int tx0,
                                    int ty0, int n, int rows, Dep &&dep, uint32_t &spans,
                                    uint32_t &kinks) {
    SpanGeom G;
    span_geom(h.flags, cf, G);
    const int bx0 = range_lo(h.bx), bx1 = range_hi(h.bx) + kRightReach;
    const int by0 = range_lo(h.by), by1 = range_hi(h.by);
    int kx0, kx1, ky0, ky1;
    axis_offsets(tx0, tx0 + n - 1, bx0, bx1, B.W, B.wrap, kx0, kx1);
    axis_offsets(ty0, ty0 + rows - 1, by0, by1, B.H, B.wrap, ky0, ky1);
    uint32_t frags = 0;
    for (int ky = ky0; ky <= ky1; ++ky) {
        const int ylo = max(ty0, by0 - ky * B.H), yhi = min(ty0 + rows - 1, by1 - ky * B.H);
        for (int kx = kx0; kx <= kx1; ++kx) {
            if (tx0 + kx * B.W > bx1 || tx0 + n - 1 + kx * B.W < bx0) continue;
            const int shift = tx0 + kx * B.W - bx0;  // record column of the tile's column 0
            // the image row in the record frame
            const double ulo = (double)(kx * B.W - bx0) - 0.5, uhi = (double)(B.W + kx * B.W - bx0) - 0.5;
            for (int y = ylo; y <= yhi; ++y) {
                const double Y = (double)(y + ky * B.H - by0) + 0.5;
                const int row = y - ty0;
                frags += row_span(G, cf, shift, Y, n, ulo, uhi, [&](int j, double v) { dep(row, j, v); }, kinks);
                ++spans;
            }
        }
    }
    return frags;
}

// All row crossings of one crease-form record in one tile (every periodic
// offset that meets it): for each crease and each tile row whose centre Y
// lies in the crease's half-open y range [y_lo, y_hi), one kink of slope
// change D at the crossing x (no step: the pyramid is continuous).  A row
// through a vertex thus meets each crease leaving it upwards, and a
// horizontal crease is never met.  Kinks left of the image are folded into
// its first two columns.  dep(row, j, v) adds v to A[row][j]; it is called
// with -2 <= j <= n + 1 and must drop the entries outside 0 <= j < n (the
// kernel keeps two padding cells on each side of a row, so that the adds
// need no test).  Returns the covered sample count (samples strictly between
// the two silhouette crossings of a row); spans counts the rows visited.
template <typename Dep>
TESS_HD inline uint32_t crease_pair(const RecHead &h, const double *cf, const BinParams &B, int tx0,
                                    int ty0, int n, int rows, Dep &&dep, uint32_t &spans,
                                    uint32_t &kinks) {
    const int m = (int)(h.flags & REC_NG_MASK);  // 3 or 4 silhouette vertices
    const int bx0 = range_lo(h.bx), bx1 = range_hi(h.bx) + kRightReach;
    const int by0 = range_lo(h.by), by1 = range_hi(h.by);
    int kx0, kx1, ky0, ky1;
    axis_offsets(tx0, tx0 + n - 1, bx0, bx1, B.W, B.wrap, kx0, kx1);
    axis_offsets(ty0, ty0 + rows - 1, by0, by1, B.H, B.wrap, ky0, ky1);
    const int jmin = -tx0;  // tile column of image column 0
    const int jlo = jmin > -2 ? jmin : -2;  // lowest deposit column (padding at -2)
    const bool left_edge = jmin > -2;  // kinks left of the tile fold into it
    int frags = 0;
    for (int ky = ky0; ky <= ky1; ++ky) {
        // record rows r (centre Y = r + 1/2) on tile rows r + rshift
        const int rshift = by0 - ky * B.H - ty0;
        const int rlo = max(-rshift, 0), rhi = min(rows - 1 - rshift, by1 - by0);
        if (rlo > rhi) continue;
        for (int kx = kx0; kx <= kx1; ++kx) {
            if (tx0 + kx * B.W > bx1 || tx0 + n - 1 + kx * B.W < bx0) continue;
            // record column of the tile's column 0
            const int shift = tx0 + kx * B.W - bx0;
            const double X0 = (double)shift + 0.5;
            // record-frame x range whose kinks reach the tile (one pixel of margin)
            const double xl = left_edge ? -1e30 : X0 - 3.0, xr = X0 + (double)n + 1.0;
            spans += (uint32_t)(rhi - rlo + 1);
            // slots 0..m-1: silhouette edge (V_k, V_k+1); slots 4..4+m-1: ridge (apex, V_k);
            // first the slots whose crease meets the tile's rows and columns
            // key of an active slot: its row count in the tile, its first and
            // last row (offsets from rlo, below 256) and the slot
            uint32_t key[8];
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                key[c] = 0u;
                const int k = c & 3;
                if (k >= m) continue;
                const int k1 = k + 1 < m ? k + 1 : 0;
                const double Px = c < 4 ? cf[k] : cf[8], Py = c < 4 ? cf[4 + k] : cf[9];
                const double Qx = c < 4 ? cf[k1] : cf[k], Qy = c < 4 ? cf[4 + k1] : cf[4 + k];
                const int r0 = max((int)ceil(fmin(Py, Qy) - 0.5), rlo);
                const int r1 = min((int)ceil(fmax(Py, Qy) - 0.5) - 1, rhi);
                if (r0 > r1 || fmax(Px, Qx) < xl) continue;
                if (fmin(Px, Qx) < xr) {
                    key[c] = ((uint32_t)(r1 - r0 + 1) << 20) | ((uint32_t)(r0 - rlo) << 12) |
                             ((uint32_t)(r1 - rlo) << 4) | (uint32_t)c;
                } else if (c < 4) {
                    // wholly right of the tile: every row counts the full width
                    frags += (cf[10 + k] > 0.0 ? -n : n) * (r1 - r0 + 1);
                }
            }
            // Longest crease first: the lanes of a wavefront step through their
            // creases together, and each step lasts as long as its longest row
            // loop, so lining up long with long and short with short shortens
            // the sum of the steps.
            sort8_desc(key);
            int nact = 0;
#pragma unroll
            for (int i = 0; i < 8; ++i) nact += key[i] != 0u ? 1 : 0;
            for (int i = 0; i < nact; ++i) {
                // take the head of the sorted queue
                const uint32_t kc = key[0];
#pragma unroll
                for (int j = 0; j < 7; ++j) key[j] = key[j + 1];
                const int c = (int)(kc & 7u);
                const int q0 = rlo + (int)((kc >> 12) & 255u), q1 = rlo + (int)((kc >> 4) & 255u);
                const int k = c & 3;
                const int k1 = k + 1 < m ? k + 1 : 0;
                const bool edge = c < 4;
                const double Px = edge ? cf[k] : cf[8], Py = edge ? cf[4 + k] : cf[9];
                const double Qx = edge ? cf[k1] : cf[k], Qy = edge ? cf[4 + k1] : cf[4 + k];
                const double bk = cf[10 + k];
                const double D = edge ? fabs(bk) : -fabs(cf[10 + (k > 0 ? k - 1 : m - 1)] - bk);
                const bool enter = bk > 0.0;
                const double sl = (Qx - Px) * fast_rcp(Qy - Py);
                int r0 = q0, r1 = q1;
                int acc = 0;  // fragment terms of this crease, before its sign
                if (Qx != Px) {
                    // keep the rows whose crossing lies in [xl, xr) (x is linear in
                    // Y, and the margins of xl and xr absorb the rounding of the
                    // reciprocal); rows cut below ya lie on the side of the bound
                    // ya comes from, rows cut above yb on the other
                    const double iv = (Qy - Py) * fast_rcp(Qx - Px);
                    double ya = Py + (xl - Px) * iv, yb = Py + (xr - Px) * iv;
                    if (ya > yb) { const double t = ya; ya = yb; yb = t; }
                    ya = fmin(fmax(ya, (double)q0 - 1.0), (double)q1 + 2.0);
                    yb = fmin(fmax(yb, (double)q0 - 1.0), (double)q1 + 2.0);
                    r0 = max(q0, (int)floor(ya - 0.5));
                    r1 = min(q1, (int)ceil(yb - 0.5));
                    // rows right of the tile count its full width
                    acc = n * (sl > 0.0 ? q1 - r1 : r0 - q0);
                }
                // the crossing u of row r in the record frame (pixel-centre
                // units, u = j at the record's column j), computed from the row
                // alone: every tile that draws it (its two entries may fall in
                // two tiles) gets the same value, and a footprint's kinks keep
                // their relative positions to the FP64 rounding of its box.
                // Fragments: an entering crossing has floor(w) + 1 samples left
                // of it in the tile frame (w = u - shift), a leaving one
                // ceil(w) (a sample on the silhouette is outside). The column
                // is taken in a frame shifted by kSampleEps, down for an
                // entering crease and up for a leaving one: k = floor(w + s)
                // and j = k + 1 is floor(w) + 1 or ceil(w), and the count is
                // max(j, 0) (jlo <= 0). Any j next to the kink gives the same
                // sum, since the deposits use the exact offset from column j:
                // with t = k - w they are D (1 + t) at j and the rest of D at
                // j + 1.
                const double s_eps = enter ? kSampleEps : -kSampleEps;
                const double cP = 0.5 - Py, xP = Px - 0.5;
                const int len = max(r1 - r0 + 1, 0);
                kinks += (uint32_t)len;
                acc += len;
                double rv = (double)r0;
                for (int r = r0; r <= r1; ++r, rv += 1.0) {
                    const int row = r + rshift;
                    const double u = fma(rv + cP, sl, xP);
                    const int k = min(max((int)floor(u + s_eps) - shift, jlo - 1), n - 1);
                    const double v1 = fma(D, (double)(k + shift) - u, D);
                    dep(row, k + 1, v1);
                    dep(row, k + 2, D - v1);
                    acc += max(k, -1);
                }
                if (edge) frags += enter ? -acc : acc;
            }
        }
    }
    return frags > 0 ? (uint32_t)frags : 0u;
}

// ------------------------------------------------- face form (depth slab)
// Upper envelope (maximum) of nl <= 4 lines a[i] + b[i] u, left to right:
// piece k follows line idx[k] up to brk[k] (the last brk is +inf). Returns
// the number of pieces.
TESS_HD inline int upper_envelope(const double a[4], const double b[4], int nl, int idx[4], double brk[4]) {
    int o[4] = {0, 1, 2, 3};
    // by slope, ascending; equal slopes: the higher line first
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = i + 1; j < 4; ++j)
            if (j < nl && (b[o[j]] < b[o[i]] || (b[o[j]] == b[o[i]] && a[o[j]] > a[o[i]]))) {
                const int t = o[i];
                o[i] = o[j];
                o[j] = t;
            }
    int ns = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (q >= nl) break;
        const int l = o[q];
        if (ns > 0 && b[idx[ns - 1]] == b[l]) continue;  // parallel and not higher
        while (ns >= 2) {
            // l overtakes the top line before the top overtakes the one below it
            const int t = idx[ns - 1], u = idx[ns - 2];
            const double xt = (a[t] - a[l]) / (b[l] - b[t]);
            const double xu = (a[u] - a[t]) / (b[t] - b[u]);
            if (xt > xu) break;
            --ns;
        }
        idx[ns++] = l;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (k < ns) brk[k] = k + 1 < ns ? (a[idx[k]] - a[idx[k + 1]]) / (b[idx[k + 1]] - b[idx[k]]) : kInf;
    return ns;
}

// One row of a face-form record: q times the chord of the ray inside the
// tetrahedron and the depth slab, t_out - t_in with t_in the largest front
// face depth (and the slab's near depth), t_out the smallest back face depth
// (and its far depth), clipped by the walls (A9 tie rule) and the image.
// Everything is evaluated in the record frame X (small numbers: a steep
// plane of an almost edge-on face keeps its precision); the tile's samples
// are u = 0..n-1 at X = X0 + u, row centre Y; break points sit at their true
// positions, pieces starting left of the image start at ulo. dep(j, v) takes
// -2 <= j <= n + 1. Returns the tile's covered samples.
template <typename Dep>
TESS_HD inline uint32_t face_row(uint32_t flags, const double *cf, const BinParams &B, int shift,
                                 double Y, int n, int jlo, double ulo, double uhi, Dep &&dep,
                                 uint32_t &kinks) {
    // evaluated in the record frame (sample u = j at the record's column j,
    // X = u + 1/2), so that every tile computes the same break points; the
    // tile's samples are u = shift .. shift + n - 1, ulo and uhi bound the
    // image row there
    constexpr double X0 = 0.5;
    const double dshift = (double)shift;
    double fa[4], fb[4], ba[4], bb[4];
    int nf = 0, nb = 0;
    double uL = ulo, uR = uhi;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        const uint32_t type = (flags >> (REC_FACE_TYPE_SHIFT + 2 * g)) & 3u;
        const double c0 = cf[3 * g], c1 = cf[3 * g + 1], c2 = cf[3 * g + 2];
        if (type == REC_FACE_WALL) {
            const bool tie = (flags >> (REC_FACE_TIE_SHIFT + g)) & 1u;
            if (c1 == 0.0) {
                const double wv = c0 + c2 * Y;
                if (!(wv > 0.0 || (wv == 0.0 && tie))) return 0;
            } else {
                // admitted samples: W > 0 (or W == 0 with the tie bit)
                const double uw = -(c0 + c2 * Y) / c1 - X0;
                if (c1 > 0.0) uL = fmax(uL, (tie ? ceil(uw) : floor(uw) + 1.0) - 0.5);
                else uR = fmin(uR, (tie ? floor(uw) : ceil(uw) - 1.0) + 0.5);
            }
        } else if (type == REC_FACE_FRONT && nf < 3) {
            fa[nf] = c0 + c2 * Y;
            fb[nf] = c1;
            ++nf;
        } else if (type == REC_FACE_BACK && nb < 3) {
            // the lower envelope of the back faces is minus the upper one of -t
            ba[nb] = -(c0 + c2 * Y);
            bb[nb] = -c1;
            ++nb;
        }
    }
    if (nf == 0 || nb == 0) return 0;
    fa[nf] = B.slab_t[0];
    fb[nf] = 0.0;
    ++nf;
    ba[nb] = -B.slab_t[1];
    bb[nb] = 0.0;
    ++nb;
    int fi[4], bi[4];
    double fbr[4], bbr[4];
    const int pf = upper_envelope(fa, fb, nf, fi, fbr);
    const int pb = upper_envelope(ba, bb, nb, bi, bbr);
    // segments of d = t_out - t_in over X, left to right, and where d > 0
    // (one interval: d is concave)
    double sA[8], sB[8], sE[8];
    int ns = 0, i = 0, k = 0;
    double zl = kInf, zr = -kInf;
#pragma unroll
    for (int it = 0; it < 8; ++it) {
        if (i >= pf || k >= pb) break;
        const double A = -ba[bi[k]] - fa[fi[i]], Bs = -bb[bi[k]] - fb[fi[i]];
        const double e = fmin(fbr[i], bbr[k]);
        const double s0 = ns > 0 ? sE[ns - 1] : -kInf;
        sA[ns] = A;
        sB[ns] = Bs;
        sE[ns] = e;
        ++ns;
        double lo = s0, hi = e;
        if (Bs > 0.0) lo = fmax(lo, -A / Bs);
        else if (Bs < 0.0) hi = fmin(hi, -A / Bs);
        else if (!(A > 0.0)) hi = lo;
        if (hi > lo) {
            zl = fmin(zl, lo);
            zr = fmax(zr, hi);
        }
        const bool ai = fbr[i] == e, ak = bbr[k] == e;
        i += ai ? 1 : 0;
        k += ak ? 1 : 0;
    }
    // the covered range, in X: d > 0, inside the walls and the image
    const double L = fmax(zl, uL + X0), R = fmin(zr, uR + X0);
    const double Lu = L - X0, Ru = R - X0;
    if (!(ceil(Ru) - floor(Lu) > 1.0)) return 0;  // no sample in (L, R)
    const double span = ceil(fmin(Ru, dshift + (double)n - 0.5)) - floor(fmax(Lu, dshift - 0.5)) - 1.0;
    const double q = cf[12];
    auto put = [&](double X, double J, double D) {
        int j = (int)floor(X - X0) + 1 - shift;  // tile column
        j = j > jlo ? j : jlo;
        j = j < n ? j : n;
        const double v1 = J + D * (((double)(j + shift) + X0) - X);
        dep(j, v1);
        dep(j + 1, D - v1);
        ++kinks;
    };
    // the pieces that hold a sample (an integer u in (lo, hi]), left to
    // right; each start is a step plus kink relative to the previous such
    // piece, so a sub-pixel piece (a face seen almost edge-on, a flat sliver)
    // becomes a step instead of two large kinks that cancel
    bool have = false;
    double pB = 0.0, pA = 0.0, last = L;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        if (t >= ns) break;
        const double s0 = t > 0 ? sE[t - 1] : -kInf;
        const double lo = fmax(s0, L), hi = fmin(sE[t], R);
        if (!(floor(hi - X0) > floor(lo - X0))) continue;
        const double A = sA[t], Bs = sB[t];
        const double J = (A + Bs * lo) - (have ? pA + pB * lo : 0.0);
        // at a zero crossing of d the first piece starts from 0
        put(lo, (!have && lo == zl) ? 0.0 : q * J, q * (Bs - pB));
        have = true;
        pA = A;
        pB = Bs;
        last = hi;
    }
    // the end: d = 0 at a zero crossing, else the value at the clip
    if (have) put(last, last == zr ? 0.0 : -q * (pA + pB * last), -q * pB);
    return span > 0.0 ? (uint32_t)span : 0u;
}

// All rows of a face-form record in one tile (every periodic offset that
// meets it).
template <typename Dep>
TESS_HD inline uint32_t face_pair(const RecHead &h, const double *cf, const BinParams &B, int tx0,
                                  int ty0, int n, int rows, Dep &&dep, uint32_t &spans, uint32_t &kinks) {
    const int bx0 = range_lo(h.bx), bx1 = range_hi(h.bx) + kRightReach;
    const int by0 = range_lo(h.by), by1 = range_hi(h.by);
    int kx0, kx1, ky0, ky1;
    axis_offsets(tx0, tx0 + n - 1, bx0, bx1, B.W, B.wrap, kx0, kx1);
    axis_offsets(ty0, ty0 + rows - 1, by0, by1, B.H, B.wrap, ky0, ky1);
    const int jmin = -tx0;
    const int jlo = jmin > -2 ? jmin : -2;
    uint32_t frags = 0;
    for (int ky = ky0; ky <= ky1; ++ky) {
        const int ylo = max(ty0, by0 - ky * B.H), yhi = min(ty0 + rows - 1, by1 - ky * B.H);
        for (int kx = kx0; kx <= kx1; ++kx) {
            if (tx0 + kx * B.W > bx1 || tx0 + n - 1 + kx * B.W < bx0) continue;
            const int shift = tx0 + kx * B.W - bx0;  // record column of the tile's column 0
            // the image row in the record frame
            const double ulo = (double)(kx * B.W - bx0) - 0.5, uhi = (double)(B.W + kx * B.W - bx0) - 0.5;
            for (int y = ylo; y <= yhi; ++y) {
                const double Y = (double)(y + ky * B.H - by0) + 0.5;
                const int row = y - ty0;
                frags += face_row(h.flags, cf, B, shift, Y, n, jlo, ulo, uhi,
                                  [&](int j, double v) { dep(row, j, v); }, kinks);
                ++spans;
            }
        }
    }
    return frags;
}

// ------------------------------------------------------ centroid splats
// A splat record's kernel values at the tile's pixel centres (every periodic
// offset that meets it), added as values: dep(row, u, w) for the tile column
// u. Returns the covered samples (W > 0); kinks counts the samples evaluated.
template <typename Dep>
TESS_HD inline uint32_t splat_pair(const RecHead &h, const double *cf, const BinParams &B, int tx0, int ty0,
                                   int n, int rows, Dep &&dep, uint32_t &spans, uint32_t &kinks) {
    const int bx0 = range_lo(h.bx), bx1 = range_hi(h.bx);
    const int by0 = range_lo(h.by), by1 = range_hi(h.by);
    int kx0, kx1, ky0, ky1;
    axis_offsets(tx0, tx0 + n - 1, bx0, bx1, B.W, B.wrap, kx0, kx1);
    axis_offsets(ty0, ty0 + rows - 1, by0, by1, B.H, B.wrap, ky0, ky1);
    const double cx = cf[0], cy = cf[1], sx = cf[2], sy = cf[3], amp = cf[4];
    uint32_t frags = 0;
    for (int ky = ky0; ky <= ky1; ++ky) {
        const int ylo = max(ty0, by0 - ky * B.H), yhi = min(ty0 + rows - 1, by1 - ky * B.H);
        for (int kx = kx0; kx <= kx1; ++kx) {
            const int ulo = max(0, bx0 - kx * B.W - tx0), uhi = min(n - 1, bx1 - kx * B.W - tx0);
            if (ulo > uhi) continue;
            const double X0 = (double)(tx0 + kx * B.W - bx0) + 0.5;
            for (int y = ylo; y <= yhi; ++y) {
                const double dy = ((double)(y + ky * B.H - by0) + 0.5 - cy) * sy;
                if (!(dy * dy < 4.0)) continue;
                const int row = y - ty0;
                ++spans;
                // the row's chord of the support circle (one column of margin)
                const double half = sqrt(4.0 - dy * dy) / sx;
                const int u0 = max(ulo, (int)floor(cx - half - X0)), u1 = min(uhi, (int)ceil(cx + half - X0));
                for (int u = u0; u <= u1; ++u) {
                    const double dx = (X0 + (double)u - cx) * sx;
                    const double q = sqrt(dx * dx + dy * dy);
                    ++kinks;
                    if (!(q < 2.0)) continue;
                    const double t = 2.0 - q;
                    const double w = q < 1.0 ? 1.0 - 1.5 * q * q + 0.75 * q * q * q : 0.25 * t * t * t;
                    dep(row, u, amp * w);
                    ++frags;
                }
            }
        }
    }
    return frags;
}

// ---------------------------------------------------- perspective camera
// A perspective record's chords at the tile's pixel centres, added as values:
// dep(row, u, q dl) for the tile column u.  The pixel at (pu, pv) on the
// window sees the half-line s (pu, pv, 1), s >= 0, in the camera frame; it is
// clipped against the four outward face planes n . y <= h (n . d == 0: the
// ray is out when h < 0, and on the plane by the orthographic raster's
// half-open rule), and dl = |(pu, pv, 1)| (s_out - s_in).  Footprints range
// from a pixel to whole tiles (next to the camera), so the pixels of the
// record's box in the tile are shared out: this call takes those with
// row-major index k = lane0, lane0 + nlanes, ...  Returns the pixels with
// dl > 0; kinks counts the pixels evaluated.  A billboard record (the
// centroid method, or beyond the hybrid's sphere) adds q |V| W(r, h) instead,
// r = z_c |(pu, pv) - (u_c, v_c)| where the ray crosses the billboard's plane.
template <typename Dep>
TESS_HD inline uint32_t persp_pair(const RecHead &h, const double *cf, const BinParams &B, int tx0, int ty0,
                                   int n, int rows, int lane0, int nlanes, Dep &&dep, uint32_t &spans,
                                   uint32_t &kinks) {
    const int x0 = max(range_lo(h.bx), tx0), x1 = min(range_hi(h.bx), tx0 + n - 1);
    const int y0 = max(range_lo(h.by), ty0), y1 = min(range_hi(h.by), ty0 + rows - 1);
    if (x0 > x1 || y0 > y1) return 0;
    const double du = B.ext_u / (double)B.W, dv = B.ext_v / (double)B.H;
    const int bw = x1 - x0 + 1, npix = bw * (y1 - y0 + 1);
    const int sy = nlanes / bw, sx = nlanes % bw;
    if (lane0 == 0) spans += (uint32_t)(y1 - y0 + 1);
    uint32_t frags = 0;
    if (h.flags & REC_SPLAT) {
        // a billboard at depth zc: the kernel at r = zc |(pu, pv) - (uc, vc)|
        const double uc = cf[0], vc = cf[1], zc = cf[2], ih = cf[3], amp = cf[4];
        int y = y0 + lane0 / bw, x = x0 + lane0 % bw;
        for (int k = lane0; k < npix; k += nlanes) {
            const double pu = -0.5 * B.ext_u + ((double)x + 0.5) * du - uc;
            const double pv = -0.5 * B.ext_v + ((double)y + 0.5) * dv - vc;
            ++kinks;
            const double s = zc * sqrt(pu * pu + pv * pv) * ih;
            if (s < 2.0) {
                const double t = 2.0 - s;
                dep(y - ty0, x - tx0, amp * (s < 1.0 ? 1.0 - 1.5 * s * s + 0.75 * s * s * s : 0.25 * t * t * t));
                ++frags;
            }
            x += sx;
            y += sy;
            if (x > x1) {
                x -= bw;
                ++y;
            }
        }
        return frags;
    }
    double nrm[4][3], off[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const int b = (a + 1) & 3, c = (a + 2) & 3, d = (a + 3) & 3;
        double e1[3], e2[3], ea[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            e1[q] = cf[3 * c + q] - cf[3 * b + q];
            e2[q] = cf[3 * d + q] - cf[3 * b + q];
            ea[q] = cf[3 * a + q] - cf[3 * b + q];
        }
        double nn[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
        if (nn[0] * ea[0] + nn[1] * ea[1] + nn[2] * ea[2] > 0.0) {
            nn[0] = -nn[0];
            nn[1] = -nn[1];
            nn[2] = -nn[2];
        }
        nrm[a][0] = nn[0];
        nrm[a][1] = nn[1];
        nrm[a][2] = nn[2];
        off[a] = nn[0] * cf[3 * b] + nn[1] * cf[3 * b + 1] + nn[2] * cf[3 * b + 2];
    }
    const double q = cf[12];
    // the chord through pixel (x, y): q |ray| (t_exit - t_entry), the ray's
    // depths where it crosses the face planes
    auto sample = [&](int x, int y) {
        const double pu = -0.5 * B.ext_u + ((double)x + 0.5) * du;
        const double pv = -0.5 * B.ext_v + ((double)y + 0.5) * dv;
        ++kinks;
        double lo = 0.0, hi = 1e300;
        bool out = false;
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            const double nd = nrm[f][0] * pu + nrm[f][1] * pv + nrm[f][2];
            if (nd > 0.0) {
                hi = fmin(hi, off[f] * fast_rcp(nd));
            } else if (nd < 0.0) {
                lo = fmax(lo, off[f] * fast_rcp(nd));
            } else if (off[f] < 0.0 ||
                       (off[f] == 0.0 && !(nrm[f][0] < 0.0 || (nrm[f][0] == 0.0 && nrm[f][1] < 0.0)))) {
                out = true;
            }
        }
        if (!out && hi > lo && hi < 1e300) {
            dep(y - ty0, x - tx0, q * ((hi - lo) * sqrt(pu * pu + pv * pv + 1.0)));
            ++frags;
        }
    };
    // (FP32: the spans only bound the columns to test, with a pixel to spare,
    // and projections within 1000 window units round to well under a pixel)
    float ex[4], ey[4];
    bool spans_ok = nlanes == 64;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const double z = cf[3 * m + 2];
        const double px = cf[3 * m] / z, py = cf[3 * m + 1] / z;
        spans_ok = spans_ok && z > 0.0 && fabs(px) < 1.0e3 && fabs(py) < 1.0e3;
        ex[m] = (float)px;
        ey[m] = (float)py;
    }
    if (spans_ok) {
        // all four vertices in front of the camera (and not near its plane):
        // the tetrahedron covers the convex hull of their projections, so a
        // row needs only the columns between its crossings with the six
        // projected edges (one pixel wider each side; the per-pixel test
        // decides).  A 16-lane group takes every fourth row of the box, its
        // lanes the row's columns (the box holds three samples per covered
        // pixel at the perspective workload).
        float sl[6];  // edge (i, j)'s x step per unit of height (a level edge: 0)
        int k = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = i + 1; j < 4; ++j, ++k) sl[k] = ey[j] != ey[i] ? (ex[j] - ex[i]) / (ey[j] - ey[i]) : 0.0f;
        const int g = lane0 >> 4, lq = lane0 & 15;
        for (int y = y0 + g; y <= y1; y += 4) {
            const float pv = (float)(-0.5 * B.ext_v + ((double)y + 0.5) * dv);
            float xl = 1e30f, xr = -1e30f;
            k = 0;
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = i + 1; j < 4; ++j, ++k) {
                    if (pv < fminf(ey[i], ey[j]) || pv > fmaxf(ey[i], ey[j])) continue;
                    const bool level = ey[j] == ey[i];
                    const float xa = level ? fminf(ex[i], ex[j]) : fmaf(pv - ey[i], sl[k], ex[i]);
                    const float xb = level ? fmaxf(ex[i], ex[j]) : xa;
                    xl = fminf(xl, xa);
                    xr = fmaxf(xr, xb);
                }
            if (!(xl <= xr)) continue;
            const double fa = ((double)xl + 0.5 * B.ext_u) / du - 0.5, fb = ((double)xr + 0.5 * B.ext_u) / du - 0.5;
            const int xa = max((int)floor(fa) - 1, x0), xb = min((int)ceil(fb) + 1, x1);
            for (int x = xa + lq; x <= xb; x += 16) sample(x, y);
        }
        return frags;
    }
    // row-major walk of the box: k -> (y, x), stepping nlanes at a time
    int y = y0 + lane0 / bw, x = x0 + lane0 % bw;
    for (int k = lane0; k < npix; k += nlanes) {
        sample(x, y);
        x += sx;
        y += sy;
        if (x > x1) {
            x -= bw;
            ++y;
        }
    }
    return frags;
}

// The rows r0 .. r1 of an edge copy whose crossing the tile holds
// (floor(fma(r, sl, base)) - shift in [-1, n - 2]; contiguous, as the
// crossing is monotone in r) as [ha, hb]: first guesses from the rows per
// column iv, then moved to the exact ends.  false: none.
TESS_HD inline bool edge_held_rows(double base, double sl, double iv, int shift, int n, int r0, int r1, int &ha,
                                   int &hb) {
    auto held = [&](int r) {
        const int kf = (int)floor(fma((double)r, sl, base)) - shift;
        return kf >= -1 && kf <= n - 2;
    };
    ha = r0;
    hb = r1;
    if (sl != 0.0) {
        double ya = ((double)(shift - 1) - base) * iv, yb = ((double)(shift + n - 1) - base) * iv;
        if (ya > yb) { const double t = ya; ya = yb; yb = t; }
        ya = fmin(fmax(ya, (double)r0), (double)r1);
        yb = fmin(fmax(yb, (double)r0), (double)r1);
        ha = (int)ya;
        hb = (int)yb;
    }
    while (ha <= hb && !held(ha)) ++ha;
    while (hb >= ha && !held(hb)) --hb;
    if (ha > hb) return false;
    while (ha > r0 && held(ha - 1)) --ha;
    while (hb < r1 && held(hb + 1)) ++hb;
    return true;
}

// The rows of an edge copy that can reach a tile's columns: those whose
// crossing lies in [shift - 3, shift + n + 1), found from the rows per
// column iv (an estimate will do: only the choice of rows depends on it,
// and it keeps a row's margin each way), within the rows [q0, q1] the tile
// holds.
TESS_HD inline void edge_copy_rows(double base, double iv, int shift, int n, int q0, int q1, int &r0, int &r1) {
    r0 = q0;
    r1 = q1;
    if (iv != 0.0) {
        double ya = ((double)(shift - 3) - base) * iv, yb = ((double)(shift + n + 1) - base) * iv;
        if (ya > yb) { const double t = ya; ya = yb; yb = t; }
        ya = fmin(fmax(ya, (double)q0 - 1.0), (double)q1 + 1.0);
        yb = fmin(fmax(yb, (double)q0 - 1.0), (double)q1 + 1.0);
        r0 = max(q0, (int)floor(ya));
        r1 = min(q1, (int)ceil(yb));
    }
}

// The seam line of a crossing at canonical position u in copy kx of an
// edge: the groups with s + kx = 1 add D (u - j), summed in A1; those with
// s + kx = 0 add -D (u - W + 2) (j + 1) when u >= W - 2, summed in A0 (the
// others add nothing).  Which of them can be nonzero follows from the
// payload's flags, taking the s = 0 sum as nonzero; A0 can act only where a
// crossing reaches the period's last two columns (in this copy the rightmost
// crossing lies before column x1 + 1 of the box, x1 = bx1 - kRightReach,
// moved by -kx W).  Returns whether the copy has a seam line; A1 and A0 its
// coefficients (the group sums read only then).
TESS_HD inline bool edge_seam_coefs(const EdgePayload &E, uint32_t eid, const BinParams &B, int tx0, int n, int kx,
                                    double &A1, double &A0) {
    const bool hasm = (E.bx & kEdgeMinus) != 0u, hasp = (E.bx & kEdgePlus) != 0u;
    const int bx1 = range_lo(E.bx) + (int)((E.bx >> 16) & kEdgeWidthMask) + kRightReach;
    const bool a1 = kx == 0 ? hasp : kx == 1 ? true : kx == 2 ? hasm : false;
    const bool a0 = kx == -1 ? hasp : kx == 0 ? true : kx == 1 ? hasm : false;
    const bool near_end = tx0 + n > B.W - 3 && bx1 - kRightReach - kx * B.W >= B.W - 3;
    A1 = 0.0;
    A0 = 0.0;
    if (!(B.seam && (a1 || (a0 && near_end)))) return false;
    double Dm = 0.0, D0 = E.D, Dp = 0.0;
    if (hasm || hasp) {
        const int64_t nedge = (int64_t)B.ntet - B.first_edge;
        Dm = B.groups[eid];
        D0 = B.groups[nedge + eid];
        Dp = B.groups[2 * nedge + eid];
    }
    A1 = kx == 0 ? Dp : kx == 1 ? D0 : kx == 2 ? Dm : 0.0;
    A0 = near_end ? (kx == -1 ? Dp : kx == 0 ? D0 : kx == 1 ? Dm : 0.0) : 0.0;
    return true;
}

// The seam line of edge copy kx (record column of the tile's column 0:
// shift, tile row of record row 0: rshift, rows r0 .. r1) without the
// fragment count, on the rows whose crossing this copy and tile hold
// (floor(u) - shift in [-1, n - 2]; contiguous, as u is monotone in r): the
// A1 part, A1 (u_c - j) with canonical position u_c = tx0 - shift + u linear
// in the tile row rho = r + rshift, as one range update a += alpha + beta
// rho, b += -A1; then the A0 part row by row where u_c >= W - 2.
template <typename Seam, typename SeamRange>
TESS_HD inline void edge_copy_seam(const EdgePayload &E, uint32_t eid, const BinParams &B, int tx0, int n, int kx,
                                   int shift, int rshift, int r0, int r1, double iv, Seam &&seam,
                                   SeamRange &&seam_range) {
    double A1, A0;
    if (!edge_seam_coefs(E, eid, B, tx0, n, kx, A1, A0)) return;
    const double sl = E.sl, base = E.base;
    int ha, hb;
    if (!edge_held_rows(base, sl, iv, shift, n, r0, r1, ha, hb)) return;
    if (A1 != 0.0) {
        const double c0 = (double)(tx0 - shift) + base - (double)rshift * sl;
        seam_range(ha + rshift, hb + rshift, A1 * c0, A1 * sl, -A1);
    }
    if (A0 != 0.0) {
        // from the end where u_c is largest, while u_c > W - 2
        const int step = sl >= 0.0 ? -1 : 1;
        const double Wm2 = (double)B.W - 2.0;
        for (int r = sl >= 0.0 ? hb : ha; r >= ha && r <= hb; r += step) {
            const double uc = (double)tx0 + (fma((double)r, sl, base) - (double)shift);
            const double near = uc - Wm2;
            if (!(near > 0.0)) break;
            seam(r + rshift, -A0 * near, -A0 * near);
        }
    }
}

// Edge form: one mesh edge's summed slope change along its projection,
// deposited on the rows whose centre lies in its half-open y range (the
// crease form's rule, so that at a vertex the edges above and below take
// the row once between them).  Nothing is folded at the image's left edge.
// Without wrap the tetrahedra behind an edge lie within the image's
// columns.  With wrap every copy of the tile takes the crossings in its
// columns, so each one's two entries land once, at its position u modulo
// the width W (u: pixel-centre units, canonical position in [-1, W - 1)).
// The running sums start at column 0, and a tetrahedron that reaches past
// the period's right end (u_T >= W - 2 in the frame that puts its left end
// in the first period) has its sums there corrected by a line a + b j added
// to the row (at columns 0 and 1 of the tile's seam cells): with d the
// slope change of one of its crossings, -d (j - u) for u_T >= W - 1 and
// -d (u - W + 2)(j + 1) for W - 2 <= u_T < W - 1 (the two agree at
// u_T = W - 1, so a crossing there may fall either way).  u_T = u + (s + kx)
// W, s the period offset of the tetrahedron's frame from the edge record's
// (Dm, D0, Dp: the slope changes summed by s = -1, 0, 1; all of D is at
// s = 0 unless the payload flags offsets), kx the tile copy.  eid: the
// edge's index among the edge records; cnt: its silhouette counts (the
// head's spare word; with COUNT only).
// Fragments: a tetrahedron's row holds (samples left of its leaving
// crossing) - (samples left of its entering crossing); each crossing adds
// its terms once, in the copy and tile holding the column right of it, in
// image columns plus (s + kx) W.  Returns the count as the bits of a signed
// 32-bit value.  COUNT = false skips the fragment count (returns 0).
//
// A row's crossing u = fma(r, sl, base) is in the record's frame and depends
// on the row alone, so a kink whose two entries fall in two tiles adds
// exactly its slope change.  Its entries: D (1 - f) at column floor(u) + 1
// and D f at floor(u) + 2, f = u - floor(u), as tile columns; the column is
// clamped so that a crossing outside the tile's columns (the rows kept are
// those whose crossing lies within a few columns of it) writes only the two
// padding cells each side, which are never read.  dep(row, j, v1, v2) adds
// v1 at tile column j and v2 at j + 1; seam(row, a, b) adds a and b to the
// row's seam line; seam_range(lo, hi, alpha, beta, gamma) adds alpha +
// beta rho to a and gamma to b on the tile rows rho in [lo, hi].
template <bool COUNT = true, bool SKIP_FIRST = false, typename Dep, typename Seam, typename SeamRange>
TESS_HD inline uint32_t edge_pair(const EdgePayload &E, uint32_t eid, uint32_t cnt, const BinParams &B, int tx0,
                                  int ty0, int n, int rows, Dep &&dep, Seam &&seam, SeamRange &&seam_range,
                                  uint32_t &kinks) {
    static_assert(!(COUNT && SKIP_FIRST), "the counting pass draws every copy itself");
    const int bx0 = range_lo(E.bx), bx1 = bx0 + (int)((E.bx >> 16) & kEdgeWidthMask) + kRightReach;
    const int by0 = range_lo(E.by), by1 = range_hi(E.by);
    int kx0, kx1, ky0, ky1;
    axis_offsets(tx0, tx0 + n - 1, bx0, bx1, B.W, B.wrap, kx0, kx1);
    axis_offsets(ty0, ty0 + rows - 1, by0, by1, B.H, B.wrap, ky0, ky1);
    const double D = E.D;
    const double sl = E.sl, base = E.base;
    // rows per column, for the rows that reach a tile's columns (only the
    // choice of rows depends on it, with a margin: an estimate will do)
    const double iv = sl != 0.0 ? fast_rcp(sl) : 0.0;
    const int ne[3] = {(int)(cnt & 7u), (int)((cnt >> 3) & 7u), (int)((cnt >> 6) & 7u)};
    const int nl[3] = {(int)((cnt >> 9) & 7u), (int)((cnt >> 12) & 7u), (int)((cnt >> 15) & 7u)};
    const bool count = cnt != 0u;
    const int nlt = nl[0] + nl[1] + nl[2], net = ne[0] + ne[1] + ne[2];
    int frags = 0;
    bool seen = false;  // a copy met already (the first one met is edge_job's)
    for (int ky = ky0; ky <= ky1; ++ky) {
        const int rshift = by0 - ky * B.H - ty0;  // tile row of record row 0
        const int q0 = max(-rshift, 0), q1 = min(rows - 1 - rshift, by1 - by0);
        if (q0 > q1) continue;
        for (int kx = kx0; kx <= kx1; ++kx) {
            if (tx0 + kx * B.W > bx1 || tx0 + n - 1 + kx * B.W < bx0) continue;
            const int shift = tx0 + kx * B.W - bx0;  // record column of the tile's column 0
            // the first copy: drawn by the caller (edge_job's copy)
            const bool first = !seen;
            seen = true;
            if (SKIP_FIRST && first) continue;
            int r0, r1;
            edge_copy_rows(base, iv, shift, n, q0, q1, r0, r1);
            kinks += (uint32_t)max(r1 - r0 + 1, 0);
            // record columns of the clamp: tile columns -3 .. n - 1
            const int klo = shift - 3, khi = shift + n - 1;
            double rv = (double)r0;
            if (!COUNT) {
                // kinks (a crossing outside the tile's columns is clamped
                // into the padding cells), then the copy's seam line
                for (int r = r0; r <= r1; ++r, rv += 1.0) {
                    const double u = fma(rv, sl, base);
                    const double fl = floor(u);
                    const int k = min(max((int)fl, klo), khi) - shift;
                    const double v1 = fma(D, fl - u, D);
                    dep(r + rshift, k + 1, v1, D - v1);
                }
                edge_copy_seam(E, eid, B, tx0, n, kx, shift, rshift, r0, r1, iv, seam, seam_range);
                continue;
            }
            double A1 = 0.0, A0 = 0.0;
            const bool seamed = edge_seam_coefs(E, eid, B, tx0, n, kx, A1, A0);
            const int wm = kx - 1, w0 = kx, wp = kx + 1;
            const int fwrap = B.W * (wm * (nl[0] - ne[0]) + w0 * (nl[1] - ne[1]) + wp * (nl[2] - ne[2]));
            const double Wm2 = (double)B.W - 2.0;
            for (int r = r0; r <= r1; ++r, rv += 1.0) {
                const int row = r + rshift;
                const double u = fma(rv, sl, base);
                const double fl = floor(u);
                const int kf = (int)fl - shift;  // the tile column left of the crossing
                const int k = min(max(kf, -3), n - 1);
                const double v1 = fma(D, fl - u, D);
                dep(row, k + 1, v1, D - v1);
                // seam line and fragment count: only where this copy and tile
                // hold the crossing
                if (kf >= -1 && kf <= n - 2) {
                    if (seamed) {
                        const double uc = (double)tx0 + (u - (double)shift);  // canonical position
                        const double near = fmax(uc - Wm2, 0.0);
                        const double a = A1 * uc - A0 * near, b = -A1 - A0 * near;
                        if (a != 0.0 || b != 0.0) seam(row, a, b);
                    }
                    if (COUNT && count) {
                        const int jl = tx0 + 1 + (int)floor(u - kSampleEps) - shift;
                        const int je = tx0 + 1 + (int)floor(u + kSampleEps) - shift;
                        frags += nlt * jl - net * je + fwrap;
                    }
                }
            }
        }
    }
    return (uint32_t)frags;
}

// The kinks of an edge's first copy in a tile (the first (ky, kx) that
// edge_pair meets), for a caller that draws them apart from the rest: row r
// of r0 .. r0 + cnt - 1 has its crossing at fma(r, sl, base), tile row
// ta + (r - r0) and column clamp floor(crossing) - shift to [-3, n - 1].
// seamed: that copy has a seam line (edge_copy_seam with copy kx and rows
// r0 .. r0 + cnt - 1 draws it); more: further copies, for edge_pair<false,
// true>, which skips exactly this one.  cnt = 0: no kinks here.
struct EdgeJob {
    double base, sl, D;
    int shift;
    int r0, ta, cnt, kx;
    bool seamed, more;
};

TESS_HD inline EdgeJob edge_job(const EdgePayload &E, const BinParams &B, int tx0, int ty0, int n, int rows,
                                uint32_t &kinks) {
    EdgeJob J;
    J.base = E.base;
    J.sl = E.sl;
    J.D = E.D;
    J.shift = 0;
    J.r0 = 0;
    J.ta = 0;
    J.cnt = 0;
    J.kx = 0;
    J.seamed = false;
    J.more = false;
    const int bx0 = range_lo(E.bx), bx1 = bx0 + (int)((E.bx >> 16) & kEdgeWidthMask) + kRightReach;
    const int by0 = range_lo(E.by), by1 = range_hi(E.by);
    int kx0, kx1, ky0, ky1;
    axis_offsets(tx0, tx0 + n - 1, bx0, bx1, B.W, B.wrap, kx0, kx1);
    axis_offsets(ty0, ty0 + rows - 1, by0, by1, B.H, B.wrap, ky0, ky1);
    const bool hasm = (E.bx & kEdgeMinus) != 0u, hasp = (E.bx & kEdgePlus) != 0u;
    const double iv = E.sl != 0.0 ? fast_rcp(E.sl) : 0.0;
    bool seen = false;
    for (int ky = ky0; ky <= ky1; ++ky) {
        const int rshift = by0 - ky * B.H - ty0;
        const int q0 = max(-rshift, 0), q1 = min(rows - 1 - rshift, by1 - by0);
        if (q0 > q1) continue;
        for (int kx = kx0; kx <= kx1; ++kx) {
            if (tx0 + kx * B.W > bx1 || tx0 + n - 1 + kx * B.W < bx0) continue;
            if (seen) {
                J.more = true;
                return J;
            }
            seen = true;
            const int shift = tx0 + kx * B.W - bx0;
            int r0, r1;
            edge_copy_rows(E.base, iv, shift, n, q0, q1, r0, r1);
            J.shift = shift;
            J.r0 = r0;
            J.ta = r0 + rshift;
            J.cnt = max(r1 - r0 + 1, 0);
            J.kx = kx;
            kinks += (uint32_t)J.cnt;
            // edge_seam_coefs's test (without reading the group sums)
            const bool a1 = kx == 0 ? hasp : kx == 1 ? true : kx == 2 ? hasm : false;
            const bool a0 = kx == -1 ? hasp : kx == 0 ? true : kx == 1 ? hasm : false;
            const bool near_end = tx0 + n > B.W - 3 && bx1 - kRightReach - kx * B.W >= B.W - 3;
            J.seamed = B.seam && (a1 || (a0 && near_end)) && J.cnt > 0;
        }
    }
    return J;
}

// One record in one tile, in whichever form its payload has.
// (A launch holds records of one kind: pyramids in crease or line form, face
// form with a depth slab, or splats; FORM selects it at compile time.)
template <int FORM, typename Dep, typename Seam>
TESS_HD inline uint32_t raster_record(const RecHead &h, const double *cf, const BinParams &B, int tx0,
                                      int ty0, int n, int rows, Dep &&dep, Seam &&seam, uint32_t &spans,
                                      uint32_t &kinks) {
    if constexpr (FORM == kFormFace) {
        return face_pair(h, cf, B, tx0, ty0, n, rows, dep, spans, kinks);
    } else if constexpr (FORM == kFormSplat) {
        return splat_pair(h, cf, B, tx0, ty0, n, rows, dep, spans, kinks);
    } else if constexpr (FORM == kFormPersp) {
        return persp_pair(h, cf, B, tx0, ty0, n, rows, 0, 1, dep, spans, kinks);
    } else {
        if (h.flags & REC_CREASE) return crease_pair(h, cf, B, tx0, ty0, n, rows, dep, spans, kinks);
        return raster_pair(h, cf, B, tx0, ty0, n, rows, dep, spans, kinks);
    }
}

}  // namespace tess
