// Internal declarations shared by the C-ABI host code and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace tess {

// Lattice and per-tetrahedron constants, all host-precomputed.
struct LatticeParams {
    const float *x, *y, *z;  // device, tracer-id order
    int32_t d[3];            // tracers per axis
    int32_t c[3];            // cubes per axis (d, or d - 1 when not periodic)
    int64_t ncubes;
    double box[3];
    int32_t periodic;
    double tet_mass;         // M / (6 cubes)
    double v0;               // mean tetrahedron volume, box volume / (6 cubes)
    double det_v0_frac;      // near-degenerate threshold (fraction of v0)
    double det_cond_k;       // conditioning threshold on the FP32 determinant (< 0: always FP64)
};

// View constants.  Pixel coordinates X = (u - u_left) * inv_du with pixel
// centres at X = ix + 1/2; likewise Y for v.
struct ViewParams {
    double rot[9];
    double center[3];
    double u_left, v_bottom;
    double inv_du, inv_dv;
    double inv_W, inv_H;     // 1 / W and 1 / H (the period tests of a wrapped image)
    double mass_px;          // 6 m * inv_du * inv_dv (density scale in pixel units)
    double crease_bmax;      // footprints with a steeper x slope keep the line form
    int32_t W, H;
    int32_t wrap;
    int32_t qpow;            // projected value q = rho^qpow (0, 1 or 2)
    // qpow == 0: the crease threshold is *qsum * bmax_per_q, qsum (device) the
    // integral of q over all tetrahedra (k_qsum); null otherwise
    const double *qsum;
    double bmax_per_q;
    int32_t slab;            // 1: only depths in [slab_t[0], slab_t[1]] count (face form)
    double slab_t[2];        // depth t = third view coordinate, R (x - c)
    int32_t splat;           // 1: centroid splats instead of the tessellation
    int32_t persp;           // 1: rays from the camera at `center` (perspective)
    int32_t hybrid;          // perspective: exact within lod_radius of the camera, billboards beyond
    double lod_radius;
    // pyramid form: 1 = the creases of tetrahedra inside the image's columns
    // are summed per mesh edge (setup writes each tetrahedron's slope change
    // per edge, and whether the edge is an entering (1) or leaving (2)
    // silhouette edge, into 36 slots per lattice vertex, slot-major; the
    // edge records carry the sums)
    int32_t edges;
    double *kinks;
    uint8_t *sil;
    // edge form: the few tetrahedra that keep their own record are numbered
    // in the order setup reaches them (*own counts them); the first own_cap
    // become records 0 .. own_cap - 1 (head and payload, the edge records
    // follow from id own_cap); the others are marked in the bit set `spill`
    // (bit 6 cube + t) and drawn by the overflow raster, which sets them up
    // again
    uint64_t own_cap;
    unsigned long long *own;
    uint32_t *spill;
};

// Record kinds of a launch (one per view): the pyramid (crease and line
// forms), the face form of a depth slab, centroid splats.
constexpr int kFormPyramid = 0, kFormFace = 1, kFormSplat = 2, kFormPersp = 3;
// the raster's instantiation for pyramids whose lists also hold edge records
constexpr int kFormEdge = 4;
__host__ __device__ inline int view_form(const ViewParams &V) {
    return V.persp ? kFormPersp : V.splat ? kFormSplat : (V.slab ? kFormFace : kFormPyramid);
}

// Screen tiling: tiles of Th rows x Tw columns (a row band when Tw >= W).
struct BinParams {
    int32_t Th, Tw;
    int32_t ntx, nty;        // tiles per axis
    int32_t W, H;
    int32_t wrap;
    int32_t seg_len;         // tetrahedra per binning segment
    int32_t nseg;
    int32_t nkey;            // work classes carried by pair ids (32), or 1: plain ids
    uint32_t ntet;           // number of records
    double slab_t[2];        // depth slab of face-form records (the view's)
    int32_t direct;          // 1: the accumulator holds values (splats, perspective), not second differences
    int32_t form;            // the records' kind (kFormPyramid, kFormFace, kFormSplat, kFormPersp)
    double ext_u, ext_v;     // the view's window (perspective: pixel rays)
    int32_t edges;           // 1: edge form (the lists hold edge records)
    uint32_t first_edge;     // edge form: id of the first edge record (6 cubes)
    int32_t seam;            // 1: edge form under wrap (tiles carry a seam line per row)
    int32_t seam_copies;     // the raster's copies of each tile row's seam line (set at launch)
    const double *groups;    // edge form: slope changes by period offset, [3][edges] (EdgePayload)
};

// Pair-list entries: the record id, with the pair's work class (0..31) in
// the bits from kClassShift up when the list carries classes
// (BinParams::nkey > 1, which needs ids below kIdMask).  kIdMask itself
// marks an empty entry.
constexpr int kClassShift = 27;
constexpr uint32_t kIdMask = (1u << kClassShift) - 1u;

// Per-call device counters (atomically accumulated).
struct DevCounters {
    unsigned long long tets, zero_volume, inverted, fp64_dets, degenerate;
    unsigned long long fragments;   // (pixel, tetrahedron) pairs with rho * dl > 0
    unsigned long long spans;       // (tetrahedron, pixel row, tile) spans rastered
    unsigned long long kinks;       // row crossings of creases (break points) evaluated
};

// Result of the binning pass, read back by the host to size the raster.
struct PlanOut {
    unsigned long long total_pairs;
    unsigned long long n_items;
    unsigned long long max_bin;
    double qsum;                    // integral of q over the tetrahedra (qpow != 1)
    unsigned long long own;         // edge form: tetrahedra that keep their own record
};

// Raster work item: a chunk of one tile's list.
struct WorkItem {
    uint64_t first;          // offset into the pair array
    uint32_t count;          // entries
    uint32_t tile;           // tile index ty * ntx + tx
};

// Per-tetrahedron raster record, stored as two arrays: the head (box and
// flags, all the binning reads) and a 128-byte FP64 payload, in pixel units
// relative to the box corner (bx0, by0).  The footprint is
//   f(p) = [all walls admit p] * max(0, min_g G_g(p)),
//   G_g(p) = a_g + b_g x + c_g y,   (x, y) = p - (bx0, by0),
// a pyramid over the projected silhouette.  Two payload forms:
//  - crease form (REC_CREASE; no walls): the silhouette vertices V_0..V_m-1
//    in cyclic order (x in c[0..3], y in c[4..7]), the apex (c[8], c[9]) and
//    the x slope b of the face over edge (V_k, V_k+1) in c[10 + k];
//  - line form: (a, b, c) of the G functions, then of the walls, in c[0..11];
//  - face form (REC_FACE; views with a depth slab): per face g, c[3g..3g+2]
//    hold its depth plane t = c0 + c1 x + c2 y (world depth over pixel
//    coordinates; front or back face) or, for a wall, its half-plane as in
//    the line form; c[12] the projected value q. The record's f(p) is q
//    times the chord inside the tetrahedron and the slab;
//  - edge form (REC_EDGE): one segment of the tetrahedral mesh, in an
//    EdgePayload (below); the head's spare word counts, by period offset, the
//    tetrahedra for which it is an entering and a leaving silhouette edge
//    (3 bits each), for the fragment count;
//  - splat (REC_SPLAT; the centroid method): centroid (c[0], c[1]), the
//    kernel's s per pixel along x and y (c[2], c[3]) and its peak amplitude
//    q |V| 10 / (7 pi h^2) (c[4]); deposited as values, not differences;
// the payload's last 16 bytes repeat the head.
struct RecHead {
    uint32_t bx;                 // pixel-centre box, x: low 16 bits x0, high 16 bits x1 (int16)
    uint32_t by;                 // y0 | y1 << 16
    uint32_t flags;
    uint32_t spare;              // crease form: row profile for scheduling (crease_profile)
};
// Box accessors (the box is stored as two packed 32-bit words).
__host__ __device__ inline uint32_t pack_range(int lo, int hi) {
    return ((uint32_t)(uint16_t)(int16_t)lo) | (((uint32_t)(uint16_t)(int16_t)hi) << 16);
}
__host__ __device__ inline int range_lo(uint32_t w) { return (int)(int16_t)(uint16_t)(w & 0xffffu); }
__host__ __device__ inline int range_hi(uint32_t w) { return (int)(int16_t)(uint16_t)(w >> 16); }
constexpr uint32_t REC_NG_MASK = 0x7u;        // number of G functions
constexpr uint32_t REC_NW_SHIFT = 3;          // number of walls (2 bits)
constexpr uint32_t REC_TIE0 = 1u << 5;        // wall 0 keeps pixels on its line
constexpr uint32_t REC_TIE1 = 1u << 6;        // wall 1 keeps pixels on its line
constexpr uint32_t REC_VALID = 1u << 7;       // some pixel centre may be covered
constexpr uint32_t REC_CREASE = 1u << 8;      // payload in crease form
constexpr uint32_t REC_FACE = 1u << 9;        // payload in face form (depth slab)
constexpr uint32_t REC_FACE_TYPE_SHIFT = 10;  // face g: 2 bits at 10 + 2 g
constexpr uint32_t REC_FACE_TIE_SHIFT = 18;   // face g's wall keeps pixels on its line
constexpr uint32_t REC_FACE_FRONT = 1u, REC_FACE_BACK = 2u, REC_FACE_WALL = 3u;
constexpr uint32_t REC_SPLAT = 1u << 22;      // payload is a centroid splat
constexpr uint32_t REC_PERSP = 1u << 23;      // payload: camera-frame vertices and q
constexpr uint32_t REC_EDGE = 1u << 24;       // a mesh edge: its summed crease (edge form)
constexpr uint32_t REC_EDGED = 1u << 25;      // a tetrahedron whose creases went to its edges

struct alignas(128) Payload {
    double c[14];
    RecHead h;  // copy of the record's head: the raster reads one 128-byte line per record
};
// Edge-form payload of an edge record (REC_EDGE), what the raster reads of
// it, in the record's frame (pixel units relative to the corner (x0, y0) of
// its box; record row r has its centre at y0 + r + 1/2, record column c at
// x0 + c): the crossing of record row r lies at column u(r) = fma(r, sl,
// base), a function of the row alone, so every tile that draws the row
// places its kink identically; D, the edge's summed slope change; the box
// (x0 and y0 .. y1 as in the head, the width x1 - x0 in 14 bits, and bits 30
// and 31 set when some of D comes from tetrahedra in a frame one period
// away, s = -1 and s = +1: the sums by s = -1, 0, 1 are then in the edge
// slots, at slot s + 1 of the slots' edge-major view, which the edge's
// vertex no longer needs once its records are written; the raster reads
// them only where a seam line needs them).  The box's rows are those
// whose centre lies in the edge's half-open y range, clipped to the image
// without wrap.  32 bytes, stored apart from the tetrahedra's payloads
// (record id - BinParams::first_edge); the head array holds box, flags and
// silhouette counts for the binning and the fragment count.
struct alignas(32) EdgePayload {
    double base, sl, D;
    uint32_t bx;  // x0 (int16) | width << 16 (14 bits) | kEdgeMinus | kEdgePlus
    uint32_t by;  // as RecHead
};
constexpr uint32_t kEdgeMinus = 1u << 30, kEdgePlus = 1u << 31;  // slope change at s = -1, +1
constexpr uint32_t kEdgeWidthMask = 0x3fffu;
static_assert(sizeof(EdgePayload) == 32, "two edges per 64 bytes");
static_assert(sizeof(RecHead) == 16, "record head");
static_assert(sizeof(Payload) == 128, "one 128-byte line per record");

// ------------------------------------------------------------ launchers
// All launchers enqueue on `stream` and return the launch status.
// Adds the integral of q over all tetrahedra (cube_qvol) into *qsum.
hipError_t launch_qsum(const LatticeParams &L, const ViewParams &V, double *qsum, hipStream_t stream);

hipError_t launch_setup(const LatticeParams &L, const ViewParams &V, RecHead *head, Payload *coef,
                        DevCounters *counters, hipStream_t stream);

// Edge records V.own_cap + tau nvert + v of every lattice vertex v from the
// kinks setup wrote (edge form).
hipError_t launch_edges(const LatticeParams &L, const ViewParams &V, RecHead *head, EdgePayload *ecoef,
                        hipStream_t stream);

hipError_t launch_count(const RecHead *head, int64_t ntet, const BinParams &B, uint32_t *counts,
                        hipStream_t stream);

// Exclusive scan of counts[n] (uint32) into base[n] (uint64); scratch must
// hold scan_scratch_elems(n) uint64.
size_t scan_scratch_elems(int64_t n);
hipError_t launch_scan(const uint32_t *counts, uint64_t *base, int64_t n, uint64_t *scratch,
                       hipStream_t stream);

// Total pairs and the longest tile list into out (n_items set to 0); when
// the total exceeds cap, *overflow (if non-null) gets bit 0 set.
hipError_t launch_totals(const uint32_t *counts, const uint64_t *base, const BinParams &B,
                         unsigned long long cap, PlanOut *out, unsigned int *overflow,
                         hipStream_t stream);

// Per-tile chunking: writes tile_items[ntiles + 1] (exclusive scan of chunk
// counts) and out->n_items; no items at all when the pairs exceed cap.
hipError_t launch_plan(const uint32_t *counts, const uint64_t *base, const BinParams &B,
                       int32_t chunk, unsigned long long cap, uint32_t *tile_items, PlanOut *out,
                       hipStream_t stream);

hipError_t launch_items(const uint64_t *base, const uint32_t *tile_items, const BinParams &B,
                        int32_t chunk, const PlanOut *plan, WorkItem *items, hipStream_t stream);

// Writes beyond pair_cap entries are dropped (memory safety if the count and
// scatter passes ever disagreed).  counts: the count pass's matrix (read only).
hipError_t launch_scatter(const RecHead *head, int64_t ntet, const BinParams &B, const uint32_t *counts,
                          const uint64_t *base, uint32_t *pairs, unsigned long long pair_cap, hipStream_t stream);

// Clears n doubles (a kernel, so that the call can sit in a captured graph).
hipError_t launch_zero(double *p, int64_t n, hipStream_t stream);

// Raster of the work items into the second-difference image acc[H][W];
// max_items blocks are launched and those beyond plan->n_items return.
// count = false: the edge form's raster skips the fragment count.
hipError_t launch_raster(const RecHead *head, const Payload *coef, const EdgePayload *ecoef, const uint32_t *pairs,
                         const WorkItem *items, uint64_t max_items, const PlanOut *plan,
                         const BinParams &B, int block, bool count, double *acc, DevCounters *counters,
                         hipStream_t stream);

// Overflow raster: when plan->total_pairs > cap (the image's tile lists were
// dropped), every record over the whole image with L2 atomics into acc;
// and (edge form) when plan->own > V.own_cap, the tetrahedra marked in
// V.spill, set up again from the lattice; otherwise the launch returns at
// once.
hipError_t launch_raster_direct(const LatticeParams &L, const ViewParams &V, const RecHead *head,
                                const Payload *coef, const EdgePayload *ecoef, const PlanOut *plan,
                                unsigned long long cap, const BinParams &B, double *acc, DevCounters *counters,
                                hipStream_t stream);

// Row-wise double prefix sum of acc -> image (FP32).
hipError_t launch_finalize(const double *acc, const BinParams &B, float *image, hipStream_t stream);

// Bytes of the allocation-free projection's scratch, a file-scope device
// array (one per device, held until the process ends).
constexpr size_t kScratchBytes = (size_t)128 << 20;
// Device address of the current device's scratch (taken once per device).
hipError_t scratch_buffer(void **ptr);

// Build-time helpers.
hipError_t launch_check_finite(const float *x, const float *y, const float *z, int64_t n,
                               unsigned long long *first_bad, hipStream_t stream);
hipError_t launch_scatter_ids(const float *x, const float *y, const float *z,
                              const uint64_t *ids, int64_t n, float *ox, float *oy, float *oz,
                              unsigned int *seen, unsigned long long *bad, hipStream_t stream);

}  // namespace tess
