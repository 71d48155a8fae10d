/*
 * tess.h -- C ABI of the MI355X phase-space-tessellation projector.
 *
 * The library renders column-density images of a dark-matter particle
 * lattice by the tetrahedral phase-space tessellation (Kaehler, Hahn & Abel,
 * arXiv:1208.3206).  Tracers sit on an implicit Lagrangian lattice (tracer
 * id = i + d0 (j + d1 k), Eq. Eqn:ID); every lattice cube is cut into six
 * tetrahedra by the connectivity table of the data-storage section; each
 * tetrahedron carries the constant mass m and density rho = m / |V|
 * (Eqs. Eqn:TetVolume, Eqn-rho_loc); a pixel accumulates, over all
 * tetrahedra its ray crosses, rho times the length of the ray inside the
 * tetrahedron (Eq. Eqn:TetProjection, the column density of the density
 * projections subsection).
 *
 * Conventions shared by every call:
 *  - Every function returns a tess_status; 0 is success.  On failure a
 *    message is available from tess_last_error() (thread-local; valid until
 *    the next call on the same thread).  No C++ exception crosses the ABI.
 *  - Device pointers are HIP device memory of the current device, owned by
 *    the caller unless stated otherwise.  Host pointers are plain host
 *    memory.  Streams are hipStream_t passed as void* (NULL = null stream).
 *  - Calls are asynchronous on the given stream unless stated otherwise.
 *  - Images are float32, row-major [height][width]; row iy holds the pixel
 *    centres v = -Sv/2 + (iy + 1/2) Sv/height, column ix the centres
 *    u = -Su/2 + (ix + 1/2) Su/width, where (u, v) are screen coordinates
 *    relative to the view centre.
 */
#ifndef TESS_H
#define TESS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TESS_OK = 0,
    TESS_EINVAL = -1,     /* an argument is invalid (message names it)          */
    TESS_ENOMEM = -2,     /* device or host allocation failed                    */
    TESS_EHIP = -3,       /* a HIP runtime call failed (message has its text)    */
    TESS_ENOTSUP = -4,    /* valid but unsupported configuration                 */
    TESS_ECAPACITY = -5,  /* a fixed capacity (tiles, image size) was exceeded   */
    TESS_ERANGE = -6      /* a value does not fit the representation in use      */
} tess_status;

/* Arithmetic of the volume determinant (Eq. Eqn:TetVolume).  The footprint
 * setup and the raster run in FP64 in both modes. */
enum {
    TESS_PREC_FP32 = 0,   /* FP32 determinant with a forward error bound; FP64 for
                             tetrahedra the bound cannot certify and for
                             near-degenerate ones (det_v0_frac, det_cond_k)      */
    TESS_PREC_FP64 = 1    /* FP64 determinant for every tetrahedron              */
};

typedef struct tess_lattice_s *tess_lattice;   /* opaque; release with tess_free */

typedef struct {
    int32_t dims[3];        /* tracers per axis (d0, d1, d2), each >= 2             */
    double box[3];          /* periodic box lengths L, > 0                           */
    int32_t periodic;       /* 1: d0 d1 d2 cubes, lattice and positions periodic
                               (corners taken modulo d, each corner moved to the
                               periodic image nearest corner 0 of its cube, offset
                               in (-L/2, L/2]); 0: (d0-1)(d1-1)(d2-1) cubes, the
                               positions used as given                           */
    double total_mass;      /* M; every tetrahedron has mass M / (6 cubes)        */
    int32_t precision;      /* TESS_PREC_FP32 or TESS_PREC_FP64                    */
    double det_v0_frac;     /* FP64 determinant when |V32| < det_v0_frac * V0,
                               V0 = box volume / (6 cubes), the mean volume       */
    double det_cond_k;      /* ... or when |V32| < det_cond_k * 2^-24 * P, where P
                               is the sum of the magnitudes of the six products
                               of the triple product (a forward error bound)      */
    int32_t copy_positions; /* 0: keep the caller's x, y, z pointers (they must
                               outlive the handle); 1: library-owned copy         */
} tess_build_desc;

/* Fills a descriptor with the defaults: periodic, unit box, total mass 1,
 * TESS_PREC_FP32, det_v0_frac 1e-6, det_cond_k 1e3, no copy.  dims are set
 * to 0 and must be filled in.  Host only; never fails for a non-null desc. */
tess_status tess_build_desc_default(tess_build_desc *desc);

/*
 * Creates a lattice handle over tracer positions (Eq. Eqn:ID).
 *   x, y, z : device float32 arrays of d0 d1 d2 positions.  Without ids they
 *             are in tracer-id order.  With ids, entry s belongs to tracer
 *             ids[s] (a permutation of 0 .. d0 d1 d2 - 1, device uint64) and
 *             the library stores an id-ordered copy (copy_positions implied).
 * Validates on the device that every position is finite and, with ids, that
 * ids is a permutation; this call synchronises `stream` once.
 * Errors: TESS_EINVAL (null pointer, dims < 2, box <= 0, mass <= 0, a
 * non-finite position -- the message names the first bad tracer id --, ids
 * not a permutation), TESS_ECAPACITY (6 x tracers at or above 2^32 - 1, the
 * 32-bit record ids), TESS_ENOMEM, TESS_EHIP.
 */
tess_status tess_build(const tess_build_desc *desc, const float *x, const float *y,
                       const float *z, const uint64_t *ids, void *stream, tess_lattice *out);

/* Releases a handle (and the positions it owns).  NULL is accepted. */
void tess_free(tess_lattice lat);

/* View: orthographic (the paper's parallel projection of the tetrahedra) or,
 * with projection = TESS_PROJECTION_PERSPECTIVE, from a camera point. */
typedef struct {
    double rot[9];          /* row-major; rows = screen u, screen v, view direction;
                               must be orthonormal (|R R^T - I| <= 1e-9)          */
    double center[3];       /* world point at the image centre; perspective: the
                               camera                                            */
    double extent[2];       /* window size (Su, Sv) in world units, > 0;
                               perspective: on the plane at unit distance along
                               the view direction                                */
    int32_t width, height;  /* pixels, 1 .. 16384 each                            */
    int32_t wrap;           /* 1: periodic image (pixel index modulo width/height);
                               requires rot to be an axis permutation with signs,
                               a periodic lattice and extent equal to the box
                               lengths along screen u and v                      */
    int32_t quantity;       /* projected per-tetrahedron value q (tess_quantity);
                               0, the zero-initialised default, is the density   */
    int32_t slab;           /* 1: only the part of each chord at depths t in
                               [slab_t[0], slab_t[1]] counts (the slab-clamped
                               fragments of the resampling section, Eqs.
                               Eqn:ResFF, Eqn:ResBF); t = third row of rot times
                               (x - center). Stacking slabs resamples the volume */
    double slab_t[2];       /* slab_t[0] < slab_t[1], finite, when slab = 1      */
    int32_t method;         /* tess_method; 0, the zero-initialised default, is
                               the exact projection of the tessellation          */
    int32_t projection;     /* tess_projection; 0, the default, is orthographic  */
    double lod_radius;      /* TESS_METHOD_HYBRID: tetrahedra whose centroid is
                               within this distance of the camera are drawn
                               exactly, the others as centroid billboards;
                               finite, >= 0                                      */
} tess_view;

/* The rays of a view.  Perspective (the camera point c of Eq. Eqn:TetSum; the
 * large-scale figure puts the camera inside the volume): the pixel at
 * (pu, pv) on the window sees the half-line c + s R^T (pu, pv, 1), s >= 0, and
 * dl is that half-line's Euclidean length inside T.  It needs wrap = 0 and
 * no slab; the raster then evaluates every covered pixel (the chord is not
 * piecewise linear along a row), so it costs per fragment.  With
 * TESS_METHOD_CENTROIDS each T is a billboard facing the view direction at
 * its centroid y_c (camera frame, drawn when z_c > 0) adding q |V| W(r, h),
 * with r the distance from y_c at which the pixel ray crosses the billboard's
 * plane, r = z_c |(pu, pv) - (x_c, y_c) / z_c|; TESS_METHOD_HYBRID draws T
 * exactly when |y_c| <= lod_radius and as a billboard otherwise (the
 * large-scale figure's sphere around the camera). */
typedef enum {
    TESS_PROJECTION_ORTHOGRAPHIC = 0,
    TESS_PROJECTION_PERSPECTIVE = 1
} tess_projection;

/* How the tetrahedra are drawn.  TESS_METHOD_CENTROIDS is the centroid
 * section's approximation: each tetrahedron T is a 2D cubic-spline kernel
 * W(r, h) = 10 / (7 pi h^2) * {1 - 3/2 s^2 + 3/4 s^3 (s < 1), 1/4 (2 - s)^3
 * (1 <= s < 2), 0}, s = r / h, at its projected centroid, with h = |V|^(1/3)
 * (the paper's size proportional to (m / rho)^(1/3), constant 1), carrying
 * q |V| (its mass for the density); not with a slab. */
typedef enum {
    TESS_METHOD_TESSELLATION = 0,
    TESS_METHOD_CENTROIDS = 1,
    TESS_METHOD_HYBRID = 2       /* perspective only: exact near, billboards far */
} tess_method;

/* The constant per-tetrahedron value q of Eq. Eqn:TetProjection, with
 * rho = m / |V| (Eq. Eqn-rho_loc): the density itself (column density), or the
 * density projections of Eq. Eqn-column-density with g = 1 (the path length
 * summed over streams: the line-of-sight integral of the stream count) and
 * g = rho^2.  Values other than the density need |V| to full precision, so
 * their determinants are all taken in FP64. */
typedef enum {
    TESS_QUANTITY_DENSITY = 0,   /* q = rho    */
    TESS_QUANTITY_UNIT = 1,      /* q = 1      */
    TESS_QUANTITY_DENSITY2 = 2   /* q = rho^2  */
} tess_quantity;

/* How plain pyramids (orthographic, no slab, the exact method) are drawn.
 * The edge form sums the creases of the tetrahedra around each mesh edge
 * before the raster (the data-storage section's cubes and six-tetrahedron
 * table form a conforming mesh); it regroups FP64 sums and changes nothing
 * else.  Other views ignore the field. */
typedef enum {
    TESS_FORM_AUTO = 0,            /* edge form when a lattice cell spans >= 1.5 pixels (wrapped image) or >= 6 */
    TESS_FORM_PER_TETRAHEDRON = 1, /* every tetrahedron drawn on its own              */
    TESS_FORM_EDGES = 2            /* edge form whenever the record ids fit 32 bits    */
} tess_form;

/* Raster parameters.  0 in a field means "choose automatically".  The image
 * is cut into tiles of tile_rows x tile_cols pixels (row bands when tile_cols
 * >= width); one raster work group holds a tile's FP64 accumulator, so
 * tile_rows * tile_cols must be <= 16384 (128 KiB of LDS). */
typedef struct {
    int32_t tile_rows;      /* 1 .. 256                                           */
    int32_t tile_cols;      /* 16 .. 16384                                        */
    int32_t chunk;          /* tile-list entries per raster work item (>= 64)     */
    int32_t block;          /* raster work-group size: 256, 512 or 1024          */
    int32_t form;           /* tess_form                                          */
    int32_t no_counts;      /* 1: with stats, the edge form's raster skips the
                               fragment count (tess_stats.fragments is then 0);
                               timings and the other counters are kept.  Without
                               stats fragments are never counted               */
    uint64_t pair_capacity; /* (record, tile) pairs the tile lists may hold; an
                               image with more is drawn by the overflow raster
                               (correct, much slower).  0: learned per lattice
                               and view shape from earlier calls' counts        */
    uint64_t workspace_limit; /* bytes of device memory the library's workspace
                               for this stream may hold after the call; a call
                               that would grow it beyond returns TESS_ENOMEM
                               before allocating anything.  0: no limit         */
    uint64_t own_capacity;  /* edge form: payloads kept for the tetrahedra that
                               keep their own record (steep or wide footprints,
                               a fraction of a percent); those beyond are set
                               up again and drawn by the overflow raster
                               (correct, slower).  0: learned per shape from
                               earlier calls (first guess: one in 64)          */
} tess_tune;

typedef struct {
    uint64_t tets;          /* tetrahedra with V != 0                             */
    uint64_t zero_volume;   /* tetrahedra skipped because V == 0                  */
    uint64_t inverted;      /* tetrahedra with V > 0 (undisplaced ones have V < 0) */
    uint64_t fp64_dets;     /* volume determinants computed in FP64               */
    uint64_t degenerate;    /* |V| < det_v0_frac * V0                             */
    uint64_t fragments;     /* (pixel, tetrahedron) pairs with rho*dl > 0         */
    uint64_t spans;         /* (tetrahedron, pixel row, tile) spans rastered by   */
                            /* per-tetrahedron records (edge records add none)    */
    uint64_t bin_pairs;     /* (tile, tetrahedron) pairs                          */
    uint32_t max_bin;       /* longest tile list                                  */
    uint32_t work_items;    /* raster work items                                  */
    int32_t tile_rows, tile_cols, chunk, block;   /* parameters used               */
    float ms;               /* device time of the call, milliseconds              */
    float setup_ms;         /* setup kernel                                       */
    float bin_ms;           /* count + scan + plan + items + scatter              */
    float raster_ms;        /* raster kernel                                      */
    float finalize_ms;      /* finalize kernel                                    */
    uint64_t kinks;         /* row crossings of creases (break points) rastered,  */
                            /* the raster's unit of arithmetic; in the edge form  */
                            /* one per (mesh edge, row, tile)                     */
    uint32_t overflow;      /* images drawn (in part) by the overflow raster: their */
                            /* pairs exceeded the pair capacity, or (edge form)    */
                            /* their tetrahedra with own records the payloads     */
    uint32_t own_records;   /* edge form: tetrahedra that kept their own record   */
                            /* (steep or wide footprints; summed over a batch)    */
} tess_stats;

/*
 * Projects the lattice onto `image` (device float32 [height][width],
 * overwritten).  Each pixel receives
 *     sum over tetrahedra T of (m / |V(T)|) * |ray(pixel centre) inside T|
 * (Eq. Eqn:TetProjection with q = rho_loc of Eq. Eqn-rho_loc), every periodic
 * image of T counted when view->wrap is set.  Tetrahedra with V == 0 are
 * skipped.
 *   tune  : host, nullable (automatic choice; see tess_tune and tess_form).
 *   stats : host, nullable; when non-null the call times its kernels with
 *           HIP events on `stream`, synchronises it and returns the counters.
 * Pixel values are sums of FP64 terms accumulated with atomics, rounded to
 * FP32 at the end: repeated calls agree to FP64 rounding, not bit for bit.
 * Plain pyramids are drawn in the form tune->form selects (automatic: the
 * edge form when a lattice cell spans at least 1.5 pixels of a periodic
 * image, or 6 pixels of a window without wrap); the edge form is not used
 * when its 13 records per lattice point would not fit 32-bit ids.
 * With stats == NULL the call only enqueues work on `stream`: it never waits
 * for the device, so it may be captured into a HIP graph once a first call
 * with the same lattice, view shape and tune has sized the workspace (the
 * workspace may grow, i.e. allocate, on a call with a new shape).  The
 * (record, tile) pair buffer is sized from the counts of earlier calls, read
 * back without waiting; an image whose pairs do not fit is drawn by the
 * overflow raster instead, with the same result.  The library owns and
 * reuses the workspace (one per device and stream); concurrent calls on one
 * handle must use different streams and output buffers.
 * Errors: TESS_EINVAL (null handle/view/image, a view that fails the checks
 * above, a tune outside its ranges), TESS_ECAPACITY (more than 32768 tiles),
 * TESS_ENOMEM, TESS_EHIP.
 */
tess_status tess_project(tess_lattice lat, const tess_view *view, const tess_tune *tune,
                         float *image, tess_stats *stats, void *stream);

/*
 * tess_project for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * image, computed by the same kernels, but every device buffer is carved out
 * of a fixed scratch array of the library (128 MiB per device, allocated
 * when the library's code is loaded on that device and held until the
 * process ends), and the call allocates nothing, device or host: no HIP
 * allocation, no events, no streams.  It only enqueues kernels on `stream`
 * and never waits for the device.  What tess_project's workspace would hold
 * for this lattice and view must fit the scratch (about a 40^3 lattice in
 * the edge form, 52^3 drawn per tetrahedron, with images of a few
 * megapixels); the (record, tile) pair list takes the rest, and an image
 * with more pairs is drawn by the overflow raster (same result, slower).
 * The caller passes the inputs (the handle) and the output (image).  Every
 * call on a device shares that device's scratch, which keeps the last
 * call's contents: calls that overlap on one device (other streams or
 * threads) race and must be ordered by the caller.  No statistics.
 *   tune : host, nullable; pair_capacity (if set) caps the pair list below
 *          what fits, no_counts is ignored.
 * Errors: as tess_project; TESS_ECAPACITY when the lattice and view do not
 * fit the scratch.
 */
tess_status tess_project_noalloc(tess_lattice lat, const tess_view *view, const tess_tune *tune,
                                 float *image, void *stream);

/*
 * Projects n_snaps lattices (same dims) through n_views views of the same
 * width/height into images laid out [n_snaps][n_views][height][width]
 * (device float32), each image the tess_project of its (snapshot, view).
 * The images' pipelines are captured once into one HIP graph, which later
 * calls with the same arguments replay on `stream` without waiting for the
 * device (stats == NULL).  Tiling and pair capacity are chosen once per
 * shape (lattice dims, image size, view kind, counts, tune): tune's fields
 * where given, otherwise the fastest candidate tiling, timed on the image
 * with the most pairs, and a capacity just above the largest pair count of
 * all the images (measured); that first call synchronises.  When the
 * environment variable TESS_TUNE_CACHE names a file, the choice is kept
 * there as JSON keyed by shape and device and read back by later processes.
 * An image whose pairs exceed the capacity is drawn by the overflow raster
 * inside the graph, and later calls capture with a larger capacity.
 * stats (host, nullable) receives the sums over all images (synchronises).
 * Errors: as tess_project; views of different sizes, snapshots of different
 * dims or periodicity -> TESS_EINVAL.
 */
tess_status tess_project_batch(const tess_lattice *snaps, int32_t n_snaps,
                               const tess_view *views, int32_t n_views,
                               const tess_tune *tune, float *images, tess_stats *stats,
                               void *stream);

/* ------------------------------------------------------------------------
 * Learned refinement.  A small network s(q) is fitted to the coarse
 * lattice's own displacement field (Lagrangian point q on the unit torus ->
 * s = x - q, minimal image, in box units):
 *   g = [sin 2 pi B q, cos 2 pi B q] (B: 64 x 3 integers, so g is periodic),
 *   four layers h = GELU(W h + b) of width 128 (exact erf GELU), s = W5 h + b5,
 * loss = mean over samples of |s - target|^2, Adam (0.9, 0.999, 1e-8) with a
 * cosine learning rate lr0 -> lr1, bf16 operands with FP32 accumulation and
 * FP32 master weights.  The r-fold sub-lattice (r d tracers per axis) is
 * then placed; coarse tracers keep their positions in every mode:
 *  - TESS_REFINE_MLP: a fine tracer gets (q + s(q)) L plus the network's
 *    residuals x - (q + s(q)) L at the corners of the coarse tetrahedron that
 *    contains q, interpolated there (so the placement is exact at the coarse
 *    tracers and the network supplies the shape between them);
 *  - TESS_REFINE_MLP_RAW: (q + s(q)) L alone;
 *  - TESS_REFINE_LINEAR: the affine map of the coarse tetrahedron containing
 *    its Lagrangian point, so the fine tetrahedra nest inside the coarse ones
 *    and the projection is unchanged.
 * The paper's tessellation (data-storage section) is the one rendered; the
 * network is an addition of this library.
 * ---------------------------------------------------------------------- */
#define TESS_MLP_PARAMS 66435   /* W1 (128x128), b1, ..., W4, b4, W5 (3x128), b5; W row = output */
#define TESS_MLP_FREQS 64

typedef enum { TESS_REFINE_LINEAR = 0, TESS_REFINE_MLP = 1, TESS_REFINE_MLP_RAW = 2 } tess_refine_mode;

typedef struct {
    int32_t r;              /* refinement factor, 1..16                            */
    int32_t mode;           /* tess_refine_mode                                    */
    int32_t steps;          /* training steps (0 with weights_in: no training)     */
    int32_t batch;          /* samples per step (drawn with replacement, counter
                               hash of seed + 1 and the step)                       */
    double rff_sigma;       /* frequencies B = rint(N(0, rff_sigma^2)) when rff_B
                               is NULL                                             */
    double lr0, lr1;        /* learning rate, cosine-decayed over the steps         */
    uint64_t seed;          /* initialisation and sampling seed                     */
    const float *rff_B;     /* host, nullable: TESS_MLP_FREQS x 3 integer values     */
    const float *weights_in;/* host, nullable: TESS_MLP_PARAMS initial parameters    */
    float *weights_out;     /* host, nullable: trained parameters                   */
} tess_refine_desc;

typedef struct {
    double loss_first, loss_last;   /* training loss at the first and last step   */
    float train_ms, infer_ms;       /* wall time of training and of placement      */
    int64_t fine_tracers;
} tess_refine_report;

/* Defaults: r 4, MLP, 10000 steps, batch 8192, sigma 8, lr 1e-2 -> 1e-5, seed 2. */
tess_status tess_refine_desc_default(tess_refine_desc *desc);

/*
 * Builds the refined lattice of a periodic coarse lattice (library-owned
 * positions; release with tess_free).  Synchronises the stream.
 * Errors: TESS_EINVAL (bad descriptor), TESS_ENOTSUP (non-periodic lattice),
 * TESS_ECAPACITY (fine lattice above 2^32 / 6 tracers), TESS_ENOMEM, TESS_EHIP.
 */
tess_status tess_refine(tess_lattice coarse, const tess_refine_desc *desc, tess_lattice *fine,
                        tess_refine_report *report, void *stream);

/*
 * One forward and backward evaluation of the network, for gradient checks.
 *   params : host, TESS_MLP_PARAMS FP32 (bf16-rounded for the products)
 *   rff_B  : host, TESS_MLP_FREQS x 3 integer-valued frequencies
 *   q, target : device, n x 3 FP32 (q on the unit torus, target in box units)
 *   loss   : host, mean over samples of |s - target|^2
 *   grad   : host, nullable, TESS_MLP_PARAMS FP32 gradient of the loss
 *   pred   : device, nullable, n x 3 predictions
 * Synchronises the stream.  Errors: TESS_EINVAL, TESS_ENOMEM, TESS_EHIP.
 */
tess_status tess_mlp_loss_grad(const float *params, const float *rff_B, const float *q,
                               const float *target, int64_t n, double *loss, float *grad,
                               float *pred, void *stream);

/*
 * The network's forward pass as tess_refine's inference runs it (one fused
 * kernel: features, hidden layers and output per 16-sample tile, bf16
 * operands rounded from the FP32 parameters, FP32 accumulation).
 *   params : host, TESS_MLP_PARAMS FP32
 *   rff_B  : host, TESS_MLP_FREQS x 3 integer-valued frequencies
 *   q      : device, n x 3 FP32 (unit torus)
 *   pred   : device, n x 3 FP32 displacements (box units), caller-owned
 * Synchronises the stream.  Errors: TESS_EINVAL (NULL, n outside 1..2^30,
 * frequencies not integers), TESS_ENOMEM, TESS_EHIP.
 */
tess_status tess_mlp_forward(const float *params, const float *rff_B, const float *q, int64_t n, float *pred,
                             void *stream);

/* One Adam update (Kingma & Ba, with bias correction), the update tess_refine
 * applies to the FP32 master parameters after each training step, for
 * checks: with m <- b1 m + (1 - b1) g and v <- b2 v + (1 - b2) g^2,
 *     params <- params - lr (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps).
 *   params, m, v : host, TESS_MLP_PARAMS FP32 each, updated in place
 *   grad         : host, TESS_MLP_PARAMS FP32
 *   step         : t >= 1
 * Runs the library's device kernel on `stream` and synchronises it.
 * Errors: TESS_EINVAL (NULL pointer, step < 1, lr, b1, b2 or eps outside
 * their ranges), TESS_ENOMEM, TESS_EHIP. */
tess_status tess_mlp_adam(float *params, float *m, float *v, const float *grad, int32_t step, double lr,
                          double beta1, double beta2, double eps, void *stream);

/* Copies a handle's tracer positions (tracer-id order; for a refined lattice
 * the placed fine tracers) into caller device arrays x, y, z of d0 d1 d2
 * floats each.  Asynchronous on `stream`.
 * Errors: TESS_EINVAL (NULL argument), TESS_EHIP. */
tess_status tess_lattice_positions(tess_lattice lat, float *x, float *y, float *z, void *stream);

/* Host-only validation of a view against a lattice description, the same
 * checks tess_project performs; usable without a GPU.  desc may be NULL
 * (then the wrap/lattice consistency checks are skipped). */
tess_status tess_check_view(const tess_view *view, const tess_build_desc *desc);

/* Host-only validation of a build descriptor; usable without a GPU. */
tess_status tess_check_build_desc(const tess_build_desc *desc);

/* Message of the last failed call on this thread ("" if none). */
const char *tess_last_error(void);

/* Library version, major * 10000 + minor * 100 + patch. */
int32_t tess_version(void);

/* sizeof of the ABI's structs as this library was compiled, for bindings to
 * check their own layouts against: which = 0 tess_build_desc, 1 tess_view,
 * 2 tess_tune, 3 tess_stats, 4 tess_refine_desc; 0 for any other value. */
uint64_t tess_struct_size(int32_t which);

#ifdef __cplusplus
}
#endif
#endif /* TESS_H */
