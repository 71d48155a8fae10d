// C ABI of the tessellation projector: argument validation, lattice handles,
// workspace management and the per-call kernel pipeline.
#include "tess_host.h"
#include "tess_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

using namespace tess;

// ----------------------------------------------------------------- errors
namespace {
thread_local std::string g_error;

bool finite3(const double *v, int n) {
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(v[i])) return false;
    return true;
}

constexpr int kMaxTiles = 32768;  // the binning keeps one 32-bit counter per tile in LDS
constexpr int kMaxTileCells = 16384;  // FP64 accumulator of one tile: 128 KiB of LDS
constexpr int kMaxSide = 16384;
}  // namespace

namespace tess {
tess_status fail(tess_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_error = buf;
    return st;
}

tess_status ok() {
    g_error.clear();
    return TESS_OK;
}

tess_lattice make_owned_lattice(const tess_build_desc &desc, float *owned, int device) {
    tess_lattice L = new tess_lattice_s();
    L->desc = desc;
    L->device = device;
    L->n = (int64_t)desc.dims[0] * desc.dims[1] * desc.dims[2];
    L->owned = owned;
    L->x = owned;
    L->y = owned + L->n;
    L->z = owned + 2 * L->n;
    return L;
}
}  // namespace tess

// ------------------------------------------------------------- workspace
namespace {
struct Workspace {
    DevBuf<RecHead> head;
    DevBuf<Payload> coef;               // the tetrahedra's payloads
    DevBuf<EdgePayload> ecoef;          // edge form: the edges' payloads
    DevBuf<double> kinks;               // edge form: 36 slope-change slots per lattice vertex
    DevBuf<uint8_t> sil;                // and their silhouette kinds
    DevBuf<uint32_t> spill;             // edge form: tetrahedra beyond the payload capacity (bits)
    DevBuf<uint32_t> counts;
    DevBuf<uint64_t> base;
    DevBuf<uint64_t> scan;
    DevBuf<uint32_t> tile_items;
    DevBuf<WorkItem> items;
    DevBuf<uint32_t> pairs;
    DevBuf<double> acc;
    DevBuf<PlanOut> plan;               // one per image of a batch
    DevBuf<DevCounters> counters;
    DevBuf<unsigned int> overflow;
    PlanOut *host_plan = nullptr;       // pinned, host_plan_cap entries
    size_t host_plan_cap = 0;
    DevCounters *host_counters = nullptr;
    unsigned int *host_overflow = nullptr;
    hipEvent_t ev[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    // pair counts of earlier calls, read back without waiting: the last
    // call's PlanOut entries are copied to fb_plan (pinned) behind fb_event;
    // the next call takes them once the event has completed
    PlanOut *fb_plan = nullptr;
    size_t fb_cap = 0;
    int fb_n = 0;
    bool fb_pending = false;
    std::string fb_key;
    hipEvent_t fb_event = nullptr;
    std::map<std::string, unsigned long long> learned;  // largest pair count seen per shape key
    std::map<std::string, unsigned long long> learned_own;  // edge form: most tetrahedra with own records
    // batch graph (captured on `capture`, replayed on the caller's stream)
    hipStream_t capture = nullptr;
    hipGraphExec_t graph = nullptr;
    std::string graph_key;
    std::mutex mu;
};

// The device buffers one projection uses (a workspace's, or views into the
// allocation-free projection's scratch).
struct Bufs {
    RecHead *head;
    Payload *coef;
    EdgePayload *ecoef;
    double *kinks;
    uint8_t *sil;
    uint32_t *spill;
    uint32_t *counts;
    uint64_t *base;
    uint64_t *scan;
    uint32_t *tile_items;
    WorkItem *items;
    uint32_t *pairs;
    double *acc;
    DevCounters *counters;
};

Bufs bufs_of(Workspace &ws) {
    return Bufs{ws.head.p, ws.coef.p, ws.ecoef.p, ws.kinks.p, ws.sil.p, ws.spill.p, ws.counts.p, ws.base.p,
                ws.scan.p, ws.tile_items.p, ws.items.p, ws.pairs.p, ws.acc.p, ws.counters.p};
}

std::mutex g_ws_mu;
std::map<std::pair<int, hipStream_t>, Workspace *> g_ws;

tess_status get_workspace(int device, hipStream_t s, Workspace **out) {
    std::lock_guard<std::mutex> lock(g_ws_mu);
    auto key = std::make_pair(device, s);
    auto it = g_ws.find(key);
    if (it != g_ws.end()) {
        *out = it->second;
        return TESS_OK;
    }
    Workspace *w = new Workspace();
    TESS_HIP(hipHostMalloc((void **)&w->host_plan, sizeof(PlanOut), hipHostMallocDefault));
    w->host_plan_cap = 1;
    TESS_HIP(hipHostMalloc((void **)&w->host_counters, sizeof(DevCounters), hipHostMallocDefault));
    TESS_HIP(hipHostMalloc((void **)&w->host_overflow, sizeof(unsigned int), hipHostMallocDefault));
    for (int i = 0; i < 6; ++i) TESS_HIP(hipEventCreate(&w->ev[i]));
    TESS_HIP(hipEventCreateWithFlags(&w->fb_event, hipEventDisableTiming));
    TESS_HIP(hipHostMalloc((void **)&w->fb_plan, sizeof(PlanOut), hipHostMallocDefault));
    w->fb_cap = 1;
    TESS_HIP(hipStreamCreateWithFlags(&w->capture, hipStreamNonBlocking));
    g_ws[key] = w;
    *out = w;
    return TESS_OK;
}
}  // namespace

// ------------------------------------------------------------ validation
extern "C" tess_status tess_build_desc_default(tess_build_desc *d) {
    if (!d) return fail(TESS_EINVAL, "tess_build_desc_default: desc is NULL");
    std::memset(d, 0, sizeof(*d));
    d->box[0] = d->box[1] = d->box[2] = 1.0;
    d->periodic = 1;
    d->total_mass = 1.0;
    d->precision = TESS_PREC_FP32;
    d->det_v0_frac = 1e-6;
    d->det_cond_k = 1e3;
    d->copy_positions = 0;
    return ok();
}

extern "C" tess_status tess_check_build_desc(const tess_build_desc *d) {
    if (!d) return fail(TESS_EINVAL, "build desc is NULL");
    for (int a = 0; a < 3; ++a) {
        if (d->dims[a] < 2) return fail(TESS_EINVAL, "dims[%d] = %d: need at least 2 tracers per axis", a, d->dims[a]);
        if (!(d->box[a] > 0) || !std::isfinite(d->box[a]))
            return fail(TESS_EINVAL, "box[%d] must be positive and finite", a);
    }
    const double n = (double)d->dims[0] * d->dims[1] * d->dims[2];
    if (6.0 * n >= 4294967295.0)  // record ids are 32-bit (and 0xffffffff marks an empty entry)
        return fail(TESS_ECAPACITY, "lattice of %.0f tracers exceeds the 32-bit tetrahedron id range", n);
    if (!(d->total_mass > 0) || !std::isfinite(d->total_mass))
        return fail(TESS_EINVAL, "total_mass must be positive and finite");
    if (d->precision != TESS_PREC_FP32 && d->precision != TESS_PREC_FP64)
        return fail(TESS_EINVAL, "precision must be TESS_PREC_FP32 or TESS_PREC_FP64");
    if (!(d->det_v0_frac >= 0) || !std::isfinite(d->det_v0_frac))
        return fail(TESS_EINVAL, "det_v0_frac must be finite and >= 0");
    if (!(d->det_cond_k >= 0) || !std::isfinite(d->det_cond_k))
        return fail(TESS_EINVAL, "det_cond_k must be finite and >= 0");
    if (d->periodic != 0 && d->periodic != 1) return fail(TESS_EINVAL, "periodic must be 0 or 1");
    return ok();
}

extern "C" tess_status tess_check_view(const tess_view *v, const tess_build_desc *d) {
    if (!v) return fail(TESS_EINVAL, "view is NULL");
    if (!finite3(v->rot, 9) || !finite3(v->center, 3) || !finite3(v->extent, 2))
        return fail(TESS_EINVAL, "view has a non-finite field");
    if (!(v->extent[0] > 0) || !(v->extent[1] > 0)) return fail(TESS_EINVAL, "view extent must be positive");
    if (v->width < 1 || v->height < 1 || v->width > kMaxSide || v->height > kMaxSide)
        return fail(TESS_EINVAL, "image %d x %d outside 1..%d", v->width, v->height, kMaxSide);
    for (int r = 0; r < 3; ++r)
        for (int s = 0; s < 3; ++s) {
            double dot = 0;
            for (int c = 0; c < 3; ++c) dot += v->rot[3 * r + c] * v->rot[3 * s + c];
            if (std::fabs(dot - (r == s ? 1.0 : 0.0)) > 1e-9)
                return fail(TESS_EINVAL, "view rotation is not orthonormal (rows %d, %d)", r, s);
        }
    if (v->wrap != 0 && v->wrap != 1) return fail(TESS_EINVAL, "wrap must be 0 or 1");
    if (v->quantity != TESS_QUANTITY_DENSITY && v->quantity != TESS_QUANTITY_UNIT &&
        v->quantity != TESS_QUANTITY_DENSITY2)
        return fail(TESS_EINVAL, "quantity must be 0 (density), 1 (unit) or 2 (density^2)");
    if (v->slab != 0 && v->slab != 1) return fail(TESS_EINVAL, "slab must be 0 or 1");
    if (v->method != TESS_METHOD_TESSELLATION && v->method != TESS_METHOD_CENTROIDS &&
        v->method != TESS_METHOD_HYBRID)
        return fail(TESS_EINVAL, "method must be 0 (tessellation), 1 (centroids) or 2 (hybrid)");
    if (v->method == TESS_METHOD_CENTROIDS && v->slab)
        return fail(TESS_EINVAL, "the centroid method takes no slab");
    if (v->projection != TESS_PROJECTION_ORTHOGRAPHIC && v->projection != TESS_PROJECTION_PERSPECTIVE)
        return fail(TESS_EINVAL, "projection must be 0 (orthographic) or 1 (perspective)");
    if (v->projection == TESS_PROJECTION_PERSPECTIVE && (v->wrap || v->slab))
        return fail(TESS_EINVAL, "a perspective view takes no wrap and no slab");
    if (v->method == TESS_METHOD_HYBRID &&
        (v->projection != TESS_PROJECTION_PERSPECTIVE || !(std::isfinite(v->lod_radius) && v->lod_radius >= 0)))
        return fail(TESS_EINVAL, "the hybrid method needs a perspective view and a finite lod_radius >= 0");
    if (v->slab && !(std::isfinite(v->slab_t[0]) && std::isfinite(v->slab_t[1]) && v->slab_t[0] < v->slab_t[1]))
        return fail(TESS_EINVAL, "slab needs finite slab_t[0] < slab_t[1]");
    if (v->wrap) {
        int axis[2];
        for (int r = 0; r < 2; ++r) {
            axis[r] = -1;
            for (int c = 0; c < 3; ++c) {
                const double e = v->rot[3 * r + c];
                if (std::fabs(std::fabs(e) - 1.0) == 0.0) axis[r] = c;
                else if (e != 0.0)
                    return fail(TESS_EINVAL, "wrap needs an axis-aligned view (row %d of rot is not a signed unit axis)", r);
            }
            if (axis[r] < 0) return fail(TESS_EINVAL, "wrap needs an axis-aligned view");
        }
        if (d) {
            if (!d->periodic) return fail(TESS_EINVAL, "wrap needs a periodic lattice");
            for (int r = 0; r < 2; ++r) {
                const double L = d->box[axis[r]];
                if (std::fabs(v->extent[r] - L) > 1e-12 * L)
                    return fail(TESS_EINVAL, "wrap needs extent[%d] == box length %.17g", r, L);
            }
        }
    }
    return ok();
}

// --------------------------------------------------------------- build
extern "C" tess_status tess_build(const tess_build_desc *desc, const float *x, const float *y,
                                  const float *z, const uint64_t *ids, void *stream,
                                  tess_lattice *out) {
    if (!out) return fail(TESS_EINVAL, "out is NULL");
    *out = nullptr;
    tess_status st = tess_check_build_desc(desc);
    if (st != TESS_OK) return st;
    if (!x || !y || !z) return fail(TESS_EINVAL, "position pointer is NULL");
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = (int64_t)desc->dims[0] * desc->dims[1] * desc->dims[2];
    int dev = 0;
    TESS_HIP(hipGetDevice(&dev));
    for (const float *p : {x, y, z}) {
        hipPointerAttribute_t attr;
        if (hipPointerGetAttributes(&attr, p) != hipSuccess || attr.type != hipMemoryTypeDevice) {
            (void)hipGetLastError();
            return fail(TESS_EINVAL, "positions must be device memory");
        }
    }
    tess_lattice L = new tess_lattice_s();
    L->desc = *desc;
    L->device = dev;
    L->n = n;
    L->owned = nullptr;
    L->x = x;
    L->y = y;
    L->z = z;
    unsigned long long *flag = nullptr;
    unsigned int *seen = nullptr;
    auto cleanup = [&](tess_status rc) {
        if (flag) (void)hipFree(flag);
        if (seen) (void)hipFree(seen);
        if (rc != TESS_OK) tess_free(L);
        return rc;
    };
    if (ids || desc->copy_positions) {
        hipError_t e = hipMalloc((void **)&L->owned, sizeof(float) * 3 * (size_t)n);
        if (e != hipSuccess) return cleanup(fail(TESS_ENOMEM, "positions copy: %s", hipGetErrorString(e)));
        float *ox = L->owned, *oy = L->owned + n, *oz = L->owned + 2 * n;
        if (hipMalloc((void **)&flag, sizeof(unsigned long long)) != hipSuccess)
            return cleanup(fail(TESS_ENOMEM, "flag allocation failed"));
        unsigned long long none = ~0ull;
        if (hipMemcpyAsync(flag, &none, sizeof(none), hipMemcpyHostToDevice, s) != hipSuccess)
            return cleanup(fail(TESS_EHIP, "flag upload failed"));
        if (ids) {
            if (hipMalloc((void **)&seen, sizeof(unsigned int) * (size_t)n) != hipSuccess)
                return cleanup(fail(TESS_ENOMEM, "id check allocation failed"));
            if (hipMemsetAsync(seen, 0, sizeof(unsigned int) * (size_t)n, s) != hipSuccess ||
                launch_scatter_ids(x, y, z, ids, n, ox, oy, oz, seen, flag, s) != hipSuccess)
                return cleanup(fail(TESS_EHIP, "id scatter failed"));
        } else {
            if (hipMemcpyAsync(ox, x, sizeof(float) * n, hipMemcpyDeviceToDevice, s) != hipSuccess ||
                hipMemcpyAsync(oy, y, sizeof(float) * n, hipMemcpyDeviceToDevice, s) != hipSuccess ||
                hipMemcpyAsync(oz, z, sizeof(float) * n, hipMemcpyDeviceToDevice, s) != hipSuccess)
                return cleanup(fail(TESS_EHIP, "position copy failed"));
        }
        unsigned long long bad = 0;
        if (hipMemcpyAsync(&bad, flag, sizeof(bad), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return cleanup(fail(TESS_EHIP, "id check readback failed"));
        if (bad != ~0ull)
            return cleanup(fail(TESS_EINVAL, "ids is not a permutation of 0..%lld (entry %llu)",
                                (long long)n - 1, bad));
        L->x = ox;
        L->y = oy;
        L->z = oz;
    }
    // every position finite
    if (!flag && hipMalloc((void **)&flag, sizeof(unsigned long long)) != hipSuccess)
        return cleanup(fail(TESS_ENOMEM, "flag allocation failed"));
    unsigned long long none = ~0ull, bad = 0;
    if (hipMemcpyAsync(flag, &none, sizeof(none), hipMemcpyHostToDevice, s) != hipSuccess ||
        launch_check_finite(L->x, L->y, L->z, n, flag, s) != hipSuccess ||
        hipMemcpyAsync(&bad, flag, sizeof(bad), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return cleanup(fail(TESS_EHIP, "finite check failed"));
    if (bad != ~0ull)
        return cleanup(fail(TESS_EINVAL, "position of tracer id %llu is not finite", bad));
    cleanup(TESS_OK);
    *out = L;
    return ok();
}

extern "C" tess_status tess_lattice_positions(tess_lattice L, float *x, float *y, float *z, void *stream) {
    if (!L || !x || !y || !z) return fail(TESS_EINVAL, "NULL argument");
    hipStream_t s = (hipStream_t)stream;
    const size_t bytes = sizeof(float) * (size_t)L->n;
    TESS_HIP(hipMemcpyAsync(x, L->x, bytes, hipMemcpyDeviceToDevice, s));
    TESS_HIP(hipMemcpyAsync(y, L->y, bytes, hipMemcpyDeviceToDevice, s));
    TESS_HIP(hipMemcpyAsync(z, L->z, bytes, hipMemcpyDeviceToDevice, s));
    return ok();
}

extern "C" void tess_free(tess_lattice L) {
    if (!L) return;
    if (L->owned) (void)hipFree(L->owned);
    delete L;
}

// ------------------------------------------------------------ projection
namespace {
void make_params(const tess_lattice_s *L, const tess_view *v, int form, LatticeParams &lp, ViewParams &vp) {
    const tess_build_desc &d = L->desc;
    lp.x = L->x;
    lp.y = L->y;
    lp.z = L->z;
    for (int a = 0; a < 3; ++a) {
        lp.d[a] = d.dims[a];
        lp.c[a] = d.periodic ? d.dims[a] : d.dims[a] - 1;
        lp.box[a] = d.box[a];
    }
    lp.ncubes = (int64_t)lp.c[0] * lp.c[1] * lp.c[2];
    lp.periodic = d.periodic;
    lp.tet_mass = d.total_mass / (6.0 * (double)lp.ncubes);
    lp.v0 = d.box[0] * d.box[1] * d.box[2] / (6.0 * (double)lp.ncubes);
    lp.det_v0_frac = d.det_v0_frac;
    lp.det_cond_k = d.precision == TESS_PREC_FP64 ? -1.0 : d.det_cond_k;
    for (int i = 0; i < 9; ++i) vp.rot[i] = v->rot[i];
    for (int i = 0; i < 3; ++i) vp.center[i] = v->center[i];
    vp.u_left = -0.5 * v->extent[0];
    vp.v_bottom = -0.5 * v->extent[1];
    vp.inv_du = v->width / v->extent[0];
    vp.inv_dv = v->height / v->extent[1];
    vp.inv_W = 1.0 / v->width;
    vp.inv_H = 1.0 / v->height;
    vp.mass_px = 6.0 * lp.tet_mass * vp.inv_du * vp.inv_dv;
    // steepest x slope a crease-form footprint may have: a kink's rounding
    // (2^-53 of its slope change) grows by up to the image width along the
    // row sums; 64 / width of the mean pixel value (all the mass in view)
    // keeps that near 1e-14 of the mean
    vp.crease_bmax = vp.mass_px * (double)lp.ncubes / ((double)v->width * (double)v->height) *
                     (64.0 / (double)v->width);
    vp.W = v->width;
    vp.H = v->height;
    vp.wrap = v->wrap;
    vp.qpow = v->quantity == TESS_QUANTITY_UNIT ? 0 : (v->quantity == TESS_QUANTITY_DENSITY2 ? 2 : 1);
    // The crease threshold in the image's own scale. q = 1: the integral of q
    // over the tetrahedra, which setup reads from the device (k_qsum fills it;
    // with many streams it far exceeds the volume). q = rho^2: the density
    // image's threshold times the mean density; the integral of rho^2 is
    // dominated by the image's peaks, where the row sums are already at their
    // noisiest, and would loosen the threshold there.
    vp.qsum = nullptr;
    vp.bmax_per_q = vp.inv_du * vp.inv_dv / ((double)v->width * (double)v->height) * (64.0 / (double)v->width);
    if (vp.qpow == 2) vp.crease_bmax *= lp.tet_mass / lp.v0;
    vp.slab = v->slab;
    vp.slab_t[0] = v->slab ? v->slab_t[0] : 0.0;
    vp.slab_t[1] = v->slab ? v->slab_t[1] : 0.0;
    vp.splat = v->method == TESS_METHOD_CENTROIDS ? 1 : 0;
    vp.persp = v->projection == TESS_PROJECTION_PERSPECTIVE ? 1 : 0;
    vp.hybrid = v->method == TESS_METHOD_HYBRID ? 1 : 0;
    vp.lod_radius = vp.hybrid ? v->lod_radius : 0.0;
    // q / rho needs |V| to full precision (the face form stores q itself, a
    // splat q |V| and |V|^(1/3))
    if (vp.qpow != 1 || vp.slab || vp.splat || vp.persp) lp.det_cond_k = -1.0;
    // Plain pyramids take the edge form when a lattice cell spans enough
    // pixels: its cost per lattice vertex (the edge records) then buys a
    // larger saving in the raster, whose work grows with the rows each
    // tetrahedron covers.  Measured on Zel'dovich lattices (128^3, 256^3):
    // periodic images favour the edge form from 1.5 pixels per cell up (1.1x
    // to 5x faster at 1.5 to 5 pixels, more beyond); windows without wrap
    // favour the per-tetrahedron form at 2 to 4 pixels per cell (rotated
    // views, 2x) and the edge form from 8 up.  tess_tune.form forces either
    // (the two give the same image up to rounding).
    const double cell_px = std::cbrt(d.box[0] * d.box[1] * d.box[2] / (double)lp.ncubes) *
                           std::sqrt(vp.inv_du * vp.inv_dv);
    const bool force_tet = form == TESS_FORM_PER_TETRAHEDRON, force_edges = form == TESS_FORM_EDGES;
    const double min_cell_px = vp.wrap ? 1.5 : 6.0;
    vp.edges = (view_form(vp) == kFormPyramid && !force_tet && (force_edges || cell_px >= min_cell_px)) ? 1 : 0;
    vp.kinks = nullptr;
    vp.sil = nullptr;
}

struct Plan {
    int Th, Tw, chunk, block;  // chunk 0: from the pair count
    int form;                  // tess_form
    unsigned long long cap;    // pair capacity; 0: learned
    int counts;                // 0: a call with stats skips the edge raster's fragment count
    unsigned long long limit;  // workspace bytes allowed after the call; 0: no limit
    unsigned long long own;    // edge form: payloads for tetrahedra with own records; 0: learned
};

// Default tiling: tiles of up to 512 columns with as many rows as the
// 128 KiB accumulator allows (at most 64). Taller tiles mean fewer (record,
// tile) pairs, narrower ones fewer columns per pair; at 2048^2, 32 x 512
// measured fastest among 8 x 1024, 16 x 1024, 32 x 512, 32 x 256 and 64 x 256.
Plan choose_plan(const tess_view *v, const tess_tune *tune) {
    Plan p;
    int Tw = (tune && tune->tile_cols) ? tune->tile_cols : std::min(v->width, 512);
    int Th = 1;
    while (Th < 64 && 2 * Th * Tw <= kMaxTileCells) Th *= 2;
    if (tune && tune->tile_rows) Th = tune->tile_rows;
    p.Th = Th;
    p.Tw = Tw;
    p.chunk = (tune && tune->chunk) ? tune->chunk : 0;
    p.block = (tune && tune->block) ? tune->block : 1024;
    p.form = tune ? tune->form : TESS_FORM_AUTO;
    p.cap = tune ? (unsigned long long)tune->pair_capacity : 0ull;
    p.counts = tune ? !tune->no_counts : 1;
    p.limit = tune ? (unsigned long long)tune->workspace_limit : 0ull;
    p.own = tune ? (unsigned long long)tune->own_capacity : 0ull;
    return p;
}

int auto_chunk(unsigned long long total_pairs) {
    // work items: a few per CU at least, each long enough to amortise its tile flush
    const unsigned long long want = total_pairs / 4096ull;
    return (int)std::min<unsigned long long>(65536ull, std::max<unsigned long long>(1024ull, want));
}

// Sizes of one image's pipeline.
struct Geometry {
    LatticeParams lp;
    ViewParams vp;
    BinParams B;
    int64_t ntet, ntiles, nmat, npix;
    int64_t stored;  // tetrahedron payloads: all (6 ncubes), or (edge form) own_cap
    int64_t spill;   // edge form: 32-bit words of the spill bit set (one spare)
};

// own_cap: edge form, the payloads for the tetrahedra that keep their own
// record (< 0: one per tetrahedron)
tess_status make_geometry(const tess_lattice_s *L, const tess_view *v, const Plan &plan, Geometry &g,
                          int64_t own_cap = -1) {
    make_params(L, v, plan.form, g.lp, g.vp);
    // records: the tetrahedra (edge form: the few that keep their own record,
    // own_cap of them), then (edge form) seven edges per lattice vertex; the
    // edge form only while all ids fit in 32 bits
    const int64_t nvert = (int64_t)g.lp.d[0] * g.lp.d[1] * g.lp.d[2];
    const int64_t ntets = 6 * g.lp.ncubes;
    if (g.vp.edges && ntets + 7 * nvert >= (int64_t)0xffffffff) g.vp.edges = 0;
    g.stored = g.vp.edges && own_cap >= 0 ? std::min<int64_t>(own_cap, ntets) : ntets;
    g.spill = g.vp.edges ? (ntets + 31) / 32 + 1 : 0;
    g.vp.own_cap = (uint64_t)g.stored;
    g.vp.own = nullptr;
    g.vp.spill = nullptr;
    g.ntet = g.stored + (g.vp.edges ? 7 * nvert : 0);
    BinParams &B = g.B;
    B.Th = plan.Th;
    B.Tw = plan.Tw;
    B.ntx = (v->width + plan.Tw - 1) / plan.Tw;
    B.nty = (v->height + plan.Th - 1) / plan.Th;
    B.W = v->width;
    B.H = v->height;
    B.wrap = v->wrap;
    g.ntiles = (int64_t)B.ntx * B.nty;
    if (g.ntiles > kMaxTiles)
        return fail(TESS_ECAPACITY, "%lld tiles of %d x %d px exceed the limit of %d; use larger tiles",
                    (long long)g.ntiles, plan.Th, plan.Tw, kMaxTiles);
    // pair ids carry a work class (pyramid records, ids below the class bits)
    B.nkey = (view_form(g.vp) == kFormPyramid && !g.vp.edges && g.ntet < (int64_t)kIdMask) ? 32 : 1;
    // binning segments: enough for the device, few enough to keep the count matrix small
    int64_t seg_len = 4096;
    while ((g.ntet + seg_len - 1) / seg_len * g.ntiles > (int64_t)64 << 20) seg_len *= 2;
    B.seg_len = (int32_t)seg_len;
    B.nseg = (int32_t)std::max<int64_t>(1, (g.ntet + seg_len - 1) / seg_len);
    B.ntet = (uint32_t)g.ntet;
    B.slab_t[0] = g.vp.slab_t[0];
    B.slab_t[1] = g.vp.slab_t[1];
    B.direct = g.vp.splat || g.vp.persp;
    B.ext_u = v->extent[0];
    B.ext_v = v->extent[1];
    B.form = view_form(g.vp);
    B.edges = g.vp.edges;
    B.first_edge = (uint32_t)g.stored;
    B.seam = g.vp.edges && v->wrap ? 1 : 0;
    B.groups = nullptr;
    g.nmat = g.ntiles * B.nseg;
    g.npix = (int64_t)B.W * B.H;
    return TESS_OK;
}

// Largest buffer sizes over the images of a call.
struct Sizes {
    int64_t records = 0, tets = 0, edges = 0, slots = 0, spill = 0, nmat = 0, ntiles = 0, npix = 0;
    void add(const Geometry &g) {
        records = std::max(records, g.ntet);
        tets = std::max(tets, g.stored);
        if (g.vp.edges) {
            edges = std::max(edges, g.ntet - g.stored);
            slots = std::max(slots, (int64_t)36 * g.lp.d[0] * g.lp.d[1] * g.lp.d[2]);
            spill = std::max(spill, g.spill);
        }
        nmat = std::max(nmat, g.nmat);
        ntiles = std::max(ntiles, g.ntiles);
        npix = std::max(npix, g.npix);
    }
};

// Bytes the workspace would hold after sizing for z and (chunk, cap), with
// n_plan PlanOut slots; checked against a tune's workspace_limit before any
// allocation.
unsigned long long max_items_for(int64_t ntiles, int chunk, unsigned long long cap);
size_t workspace_bytes_after(const Workspace &ws, const Sizes &z, int chunk, unsigned long long cap, size_t n_plan) {
    size_t b = 0;
    b += ws.head.bytes_after((size_t)z.records) + ws.coef.bytes_after((size_t)z.tets);
    if (z.edges)
        b += ws.ecoef.bytes_after((size_t)z.edges) + ws.kinks.bytes_after((size_t)z.slots) +
             ws.sil.bytes_after((size_t)z.slots) + ws.spill.bytes_after((size_t)z.spill);
    else
        b += ws.ecoef.cap * sizeof(EdgePayload) + ws.kinks.cap * sizeof(double) + ws.sil.cap +
             ws.spill.cap * sizeof(uint32_t);
    b += ws.counts.bytes_after((size_t)z.nmat) + ws.base.bytes_after((size_t)z.nmat) +
         ws.scan.bytes_after(scan_scratch_elems(z.nmat)) + ws.tile_items.bytes_after((size_t)z.ntiles + 1) +
         ws.acc.bytes_after((size_t)z.npix) + ws.counters.bytes_after(1) + ws.overflow.bytes_after(1) +
         ws.plan.bytes_after(n_plan);
    b += ws.items.bytes_after((size_t)std::max<unsigned long long>(max_items_for(z.ntiles, chunk, cap), 1)) +
         ws.pairs.bytes_after((size_t)std::max<unsigned long long>(cap, 1));
    return b;
}

tess_status check_limit(const Workspace &ws, const Plan &plan, const Sizes &z, int chunk, unsigned long long cap,
                        size_t n_plan) {
    if (!plan.limit) return TESS_OK;
    const size_t b = workspace_bytes_after(ws, z, chunk, cap, n_plan);
    if (b > plan.limit)
        return fail(TESS_ENOMEM, "the workspace would hold %.1f MiB, above tune.workspace_limit (%.1f MiB)",
                    b / 1048576.0, plan.limit / 1048576.0);
    return TESS_OK;
}

tess_status ensure_front(Workspace &ws, const Sizes &z) {
    TESS_HIP(ws.head.ensure((size_t)z.records));
    TESS_HIP(ws.coef.ensure((size_t)z.tets));
    if (z.edges) {
        TESS_HIP(ws.ecoef.ensure((size_t)z.edges));
        TESS_HIP(ws.kinks.ensure((size_t)z.slots));
        TESS_HIP(ws.sil.ensure((size_t)z.slots));
        TESS_HIP(ws.spill.ensure((size_t)z.spill));
    }
    TESS_HIP(ws.counts.ensure((size_t)z.nmat));
    TESS_HIP(ws.base.ensure((size_t)z.nmat));
    TESS_HIP(ws.scan.ensure(scan_scratch_elems(z.nmat)));
    TESS_HIP(ws.tile_items.ensure((size_t)z.ntiles + 1));
    TESS_HIP(ws.acc.ensure((size_t)z.npix));
    TESS_HIP(ws.counters.ensure(1));
    TESS_HIP(ws.overflow.ensure(1));
    return TESS_OK;
}

unsigned long long max_items_for(int64_t ntiles, int chunk, unsigned long long cap) {
    return cap / (unsigned long long)chunk + (unsigned long long)ntiles;
}

tess_status ensure_back(Workspace &ws, int64_t ntiles, int chunk, unsigned long long cap) {
    TESS_HIP(ws.items.ensure((size_t)std::max<unsigned long long>(max_items_for(ntiles, chunk, cap), 1)));
    TESS_HIP(ws.pairs.ensure((size_t)std::max<unsigned long long>(cap, 1)));
    return TESS_OK;
}

// Setup of one image; for q = 1 first the integral of q into slot->qsum.
tess_status enqueue_setup(const Geometry &g, const Bufs &b, PlanOut *slot, hipStream_t s) {
    ViewParams vp = g.vp;
    if (vp.qpow == 0 && !vp.slab && !vp.splat && !vp.persp) {
        TESS_HIP(launch_zero(&slot->qsum, 1, s));
        TESS_HIP(launch_qsum(g.lp, vp, &slot->qsum, s));
        vp.qsum = &slot->qsum;
    }
    vp.kinks = b.kinks;
    vp.sil = b.sil;
    TESS_HIP(launch_zero((double *)&slot->own, 1, s));  // (+0.0: all bits zero)
    if (vp.edges) {
        // the numbered records start invalid (setup fills as many as it
        // finds), the spill set empty
        vp.own = &slot->own;
        vp.spill = b.spill;
        static_assert(sizeof(RecHead) == 2 * sizeof(double), "head as two doubles");
        TESS_HIP(launch_zero((double *)b.head, 2 * g.stored, s));
        TESS_HIP(launch_zero((double *)b.spill, g.spill / 2, s));
    }
    TESS_HIP(launch_setup(g.lp, vp, b.head, b.coef, b.counters, s));
    if (vp.edges) TESS_HIP(launch_edges(g.lp, vp, b.head, b.ecoef, s));
    return TESS_OK;
}

// Setup, count, scan and totals of one image (no host synchronisation);
// the totals flag *overflow when the pairs exceed cap.
tess_status enqueue_front(const Geometry &g, const Bufs &b, PlanOut *slot, unsigned long long cap,
                          unsigned int *overflow, hipStream_t s) {
    tess_status st = enqueue_setup(g, b, slot, s);
    if (st != TESS_OK) return st;
    TESS_HIP(launch_count(b.head, g.ntet, g.B, b.counts, s));
    TESS_HIP(launch_scan(b.counts, b.base, g.nmat, b.scan, s));
    TESS_HIP(launch_totals(b.counts, b.base, g.B, cap, slot, overflow, s));
    return TESS_OK;
}

// Work items, scatter, raster and finalize of one image into `image`, for at
// most `cap` pairs (the buffers hold that many); an image with more pairs
// gets no work items and is drawn by the overflow raster.
tess_status enqueue_back(const Geometry &g, const Plan &plan, int chunk, unsigned long long cap, bool count,
                         const Bufs &b, PlanOut *slot, float *image, hipStream_t s, hipEvent_t after_bin,
                         hipEvent_t after_raster) {
    TESS_HIP(launch_plan(b.counts, b.base, g.B, chunk, cap, b.tile_items, slot, s));
    TESS_HIP(launch_items(b.base, b.tile_items, g.B, chunk, slot, b.items, s));
    TESS_HIP(launch_scatter(b.head, g.ntet, g.B, b.counts, b.base, b.pairs, cap, s));
    TESS_HIP(launch_zero(b.acc, g.npix, s));
    if (after_bin) TESS_HIP(hipEventRecord(after_bin, s));
    BinParams B = g.B;
    B.groups = b.kinks;  // the edge records' sums by period offset (written over the slots)
    TESS_HIP(launch_raster(b.head, b.coef, b.ecoef, b.pairs, b.items, max_items_for(g.ntiles, chunk, cap), slot,
                           B, plan.block, count, b.acc, b.counters, s));
    ViewParams vp = g.vp;
    vp.kinks = b.kinks;
    vp.sil = b.sil;
    vp.own = &slot->own;
    vp.spill = b.spill;
    TESS_HIP(launch_raster_direct(g.lp, vp, b.head, b.coef, b.ecoef, slot, cap, B, b.acc, b.counters, s));
    if (after_raster) TESS_HIP(hipEventRecord(after_raster, s));
    TESS_HIP(launch_finalize(b.acc, g.B, image, s));
    return TESS_OK;
}

void fill_stats(tess_stats *stats, const DevCounters &c, const Plan &plan, int chunk) {
    stats->tets = c.tets;
    stats->zero_volume = c.zero_volume;
    stats->inverted = c.inverted;
    stats->fp64_dets = c.fp64_dets;
    stats->degenerate = c.degenerate;
    stats->fragments = c.fragments;
    stats->spans = c.spans;
    stats->kinks = c.kinks;
    stats->tile_rows = plan.Th;
    stats->tile_cols = plan.Tw;
    stats->chunk = chunk;
    stats->block = plan.block;
}

// ------------------------------------------------------ pair capacities
// The (record, tile) pair count is known only on the device.  Calls size the
// pair buffer from the counts of earlier calls with the same shape, which
// come back through pinned memory behind an event that is polled, never
// waited for; until one is known, from a first guess.  An image that does
// not fit is still drawn (the overflow raster), and its count raises the
// capacity of later calls.
std::string count_key(const Geometry &g) {
    char buf[256];
    snprintf(buf, sizeof(buf), "%d:%d:%d:%d|%dx%d:%d:%d:%d:%d:%d|%dx%d", g.lp.d[0], g.lp.d[1], g.lp.d[2], g.lp.periodic,
             g.B.W, g.B.H, g.B.wrap, g.B.form, g.B.edges, g.vp.qpow, g.vp.hybrid, g.B.Th, g.B.Tw);
    return buf;
}

unsigned long long capacity_for(unsigned long long most) { return most + most / 8 + 4096; }

// Edge form: payloads for the tetrahedra that keep their own record (steep
// or wide footprints): from the most seen for this shape, else a first guess
// of one in 64 (measured: 0.2 % on a 64^3 lattice at 8 pixels per cell);
// those beyond are drawn by the overflow raster and raise the next call's.
int64_t own_capacity(const Workspace &ws, const Geometry &g0, const std::string &key, const Plan &plan) {
    const int64_t ntets = 6 * g0.lp.ncubes;
    if (plan.own) return std::min<int64_t>((int64_t)plan.own, ntets);
    auto it = ws.learned_own.find(key);
    const int64_t want = it != ws.learned_own.end() ? (int64_t)capacity_for(it->second) : ntets / 64 + 65536;
    return std::min<int64_t>(want, ntets);
}

// First guess without any count: four pairs per record, seven in the edge
// form, whose records are nearly all edges (the stress workload at 2048^2
// with 32 x 512 tiles has 6.0 pairs per edge), within [2^20, 2^31].
unsigned long long first_guess(const Geometry &g) {
    const unsigned long long want = (g.vp.edges ? 7ull : 4ull) * (unsigned long long)g.ntet;
    return std::min<unsigned long long>(std::max<unsigned long long>(want, 1ull << 20), 1ull << 31);
}

bool capturing(hipStream_t s) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone;
}

// Takes the counts of the last call if they have arrived (never waits).
void take_feedback(Workspace &ws, hipStream_t s) {
    if (!ws.fb_pending || capturing(s)) return;
    if (hipEventQuery(ws.fb_event) != hipSuccess) {
        (void)hipGetLastError();  // not ready (or failed): try again on a later call
        return;
    }
    unsigned long long most = 0, own = 0;
    for (int k = 0; k < ws.fb_n; ++k) {
        most = std::max<unsigned long long>(most, ws.fb_plan[k].total_pairs);
        own = std::max<unsigned long long>(own, ws.fb_plan[k].own);
    }
    unsigned long long &m = ws.learned[ws.fb_key];
    m = std::max(m, most);
    if (own) {
        unsigned long long &o = ws.learned_own[ws.fb_key];
        o = std::max(o, own);
    }
    ws.fb_pending = false;
}

// Copies n PlanOut entries to the pinned feedback area behind an event.
tess_status give_feedback(Workspace &ws, const PlanOut *plan, int n, const std::string &key, hipStream_t s) {
    if (ws.fb_pending || capturing(s)) return TESS_OK;
    if (ws.fb_cap < (size_t)n) {
        TESS_HIP(hipHostFree(ws.fb_plan));
        ws.fb_plan = nullptr;
        ws.fb_cap = 0;
        TESS_HIP(hipHostMalloc((void **)&ws.fb_plan, sizeof(PlanOut) * (size_t)n, hipHostMallocDefault));
        ws.fb_cap = (size_t)n;
    }
    TESS_HIP(hipMemcpyAsync(ws.fb_plan, plan, sizeof(PlanOut) * (size_t)n, hipMemcpyDeviceToHost, s));
    TESS_HIP(hipEventRecord(ws.fb_event, s));
    ws.fb_n = n;
    ws.fb_key = key;
    ws.fb_pending = true;
    return TESS_OK;
}

// One image.  Without stats nothing waits for the device.
tess_status project_impl(const tess_lattice_s *L, const tess_view *v, const Plan &plan, float *image,
                         tess_stats *stats, hipStream_t s, Workspace &ws) {
    Geometry g;
    tess_status st = make_geometry(L, v, plan, g);
    if (st != TESS_OK) return st;
    take_feedback(ws, s);
    const std::string key = count_key(g);
    if (g.vp.edges) {
        st = make_geometry(L, v, plan, g, own_capacity(ws, g, key, plan));
        if (st != TESS_OK) return st;
    }
    Sizes z;
    z.add(g);
    auto it = ws.learned.find(key);
    const bool known = it != ws.learned.end();
    const unsigned long long cap = plan.cap ? plan.cap : (known ? capacity_for(it->second) : first_guess(g));
    const int chunk = plan.chunk ? plan.chunk : auto_chunk(known ? it->second : cap / 2);
    st = check_limit(ws, plan, z, chunk, cap, 1);
    if (st != TESS_OK) return st;
    st = ensure_front(ws, z);
    if (st != TESS_OK) return st;
    TESS_HIP(ws.plan.ensure(1));
    st = ensure_back(ws, g.ntiles, chunk, cap);
    if (st != TESS_OK) return st;
    if (stats) TESS_HIP(hipEventRecord(ws.ev[0], s));
    TESS_HIP(launch_zero((double *)ws.counters.p, sizeof(DevCounters) / sizeof(double), s));
    const Bufs b = bufs_of(ws);
    st = enqueue_setup(g, b, ws.plan.p, s);
    if (st != TESS_OK) return st;
    if (stats) TESS_HIP(hipEventRecord(ws.ev[1], s));
    TESS_HIP(launch_count(ws.head.p, g.ntet, g.B, ws.counts.p, s));
    TESS_HIP(launch_scan(ws.counts.p, ws.base.p, g.nmat, ws.scan.p, s));
    TESS_HIP(launch_totals(ws.counts.p, ws.base.p, g.B, cap, ws.plan.p, nullptr, s));
    st = enqueue_back(g, plan, chunk, cap, stats != nullptr && plan.counts, b, ws.plan.p, image, s,
                      stats ? ws.ev[2] : nullptr, stats ? ws.ev[3] : nullptr);
    if (st != TESS_OK) return st;
    if (!stats) return give_feedback(ws, ws.plan.p, 1, key, s);
    TESS_HIP(hipEventRecord(ws.ev[4], s));
    TESS_HIP(hipMemcpyAsync(ws.host_counters, ws.counters.p, sizeof(DevCounters), hipMemcpyDeviceToHost, s));
    TESS_HIP(hipMemcpyAsync(ws.host_plan, ws.plan.p, sizeof(PlanOut), hipMemcpyDeviceToHost, s));
    TESS_HIP(hipStreamSynchronize(s));
    float ms = 0, t_setup = 0, t_bin = 0, t_raster = 0, t_fin = 0;
    TESS_HIP(hipEventElapsedTime(&ms, ws.ev[0], ws.ev[4]));
    TESS_HIP(hipEventElapsedTime(&t_setup, ws.ev[0], ws.ev[1]));
    TESS_HIP(hipEventElapsedTime(&t_bin, ws.ev[1], ws.ev[2]));
    TESS_HIP(hipEventElapsedTime(&t_raster, ws.ev[2], ws.ev[3]));
    TESS_HIP(hipEventElapsedTime(&t_fin, ws.ev[3], ws.ev[4]));
    const PlanOut &P = *ws.host_plan;
    unsigned long long &m = ws.learned[key];
    m = std::max<unsigned long long>(m, P.total_pairs);
    if (g.vp.edges) {
        unsigned long long &o = ws.learned_own[key];
        o = std::max<unsigned long long>(o, P.own);
    }
    fill_stats(stats, *ws.host_counters, plan, chunk);
    stats->bin_pairs = P.total_pairs;
    stats->max_bin = (uint32_t)std::min<unsigned long long>(P.max_bin, 0xffffffffull);
    stats->work_items = (uint32_t)P.n_items;
    stats->overflow = P.total_pairs > cap || (g.vp.edges && P.own > g.vp.own_cap) ? 1u : 0u;
    stats->own_records = (uint32_t)std::min<unsigned long long>(P.own, 0xffffffffull);
    stats->ms = ms;
    stats->setup_ms = t_setup;
    stats->bin_ms = t_bin;
    stats->raster_ms = t_raster;
    stats->finalize_ms = t_fin;
    return TESS_OK;
}

tess_status check_project_args(tess_lattice L, const tess_view *v, const tess_tune *tune, float *image) {
    if (!L) return fail(TESS_EINVAL, "lattice handle is NULL");
    if (!image) return fail(TESS_EINVAL, "image is NULL");
    tess_status st = tess_check_view(v, &L->desc);
    if (st != TESS_OK) return st;
    if (tune) {
        if (tune->tile_rows < 0 || tune->tile_rows > 256)
            return fail(TESS_EINVAL, "tune.tile_rows must be 0 (automatic) or 1..256");
        if (tune->tile_cols != 0 && (tune->tile_cols < 16 || tune->tile_cols > kMaxTileCells))
            return fail(TESS_EINVAL, "tune.tile_cols must be 0 (automatic) or 16..%d", kMaxTileCells);
        const Plan p = choose_plan(v, tune);
        if ((int64_t)p.Th * p.Tw > kMaxTileCells)
            return fail(TESS_EINVAL, "tile of %d x %d pixels exceeds %d cells", p.Th, p.Tw, kMaxTileCells);
        if (tune->chunk != 0 && tune->chunk < 64) return fail(TESS_EINVAL, "tune.chunk must be 0 or >= 64");
        if (tune->block != 0 && tune->block != 256 && tune->block != 512 && tune->block != 1024)
            return fail(TESS_EINVAL, "tune.block must be 0, 256, 512 or 1024");
        if (tune->form != TESS_FORM_AUTO && tune->form != TESS_FORM_PER_TETRAHEDRON && tune->form != TESS_FORM_EDGES)
            return fail(TESS_EINVAL, "tune.form must be 0 (automatic), 1 (per tetrahedron) or 2 (edges)");
        if (tune->no_counts != 0 && tune->no_counts != 1) return fail(TESS_EINVAL, "tune.no_counts must be 0 or 1");
    }
    return TESS_OK;
}

tess_status lock_workspace(tess_lattice L, hipStream_t s, Workspace **ws) {
    int dev = 0;
    TESS_HIP(hipGetDevice(&dev));
    if (dev != L->device) return fail(TESS_EINVAL, "lattice lives on device %d, current device is %d", L->device, dev);
    return get_workspace(dev, s, ws);
}

// ---------------------------------------------------------------- batches
// Raster parameters and pair capacity chosen for a batch shape, kept for
// later calls with the same lattice and image shape, in this process and,
// when the environment variable TESS_TUNE_CACHE names a file, in that JSON
// file (keyed by the shape and the device).
struct Tuned {
    Plan plan;
    int chunk;
    unsigned long long cap;
};
std::mutex g_tune_mu;
std::map<std::string, Tuned> g_tuned;

std::string shape_key(const tess_lattice_s *L, const tess_view *v, int n_snaps, int n_views, const tess_tune *tune) {
    char buf[384];
    int dev = 0;
    hipDeviceProp_t prop;
    std::memset(&prop, 0, sizeof(prop));
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) (void)hipGetLastError();
    std::string arch(prop.gcnArchName);
    arch = arch.substr(0, arch.find(':'));
    snprintf(buf, sizeof(buf), "%s/%dcu|%d:%d:%d:%d|%dx%d:%d:%d:%d:%d:%d|%d:%d|tune %d %d %d %d %d %llu %llu",
             arch.c_str(), prop.multiProcessorCount, L->desc.dims[0], L->desc.dims[1], L->desc.dims[2],
             L->desc.periodic, v->width, v->height, v->wrap, v->quantity, v->slab, v->method, v->projection,
             n_snaps, n_views, tune ? tune->tile_rows : 0, tune ? tune->tile_cols : 0, tune ? tune->chunk : 0,
             tune ? tune->block : 0, tune ? tune->form : 0,
             tune ? (unsigned long long)tune->pair_capacity : 0ull,
             tune ? (unsigned long long)tune->own_capacity : 0ull);
    return buf;
}

// ---- the JSON tune cache: one object per line inside "entries", e.g.
// {"key": "...", "tile_rows": 64, "tile_cols": 256, "chunk": 1024, "block": 1024, "form": 0, "pair_capacity": 123}
const char *tune_cache_path() {
    const char *p = getenv("TESS_TUNE_CACHE");
    return (p && p[0]) ? p : nullptr;
}

bool json_string(const std::string &line, const char *field, std::string &out) {
    const std::string pat = std::string("\"") + field + "\": \"";
    const size_t a = line.find(pat);
    if (a == std::string::npos) return false;
    const size_t b = line.find('"', a + pat.size());
    if (b == std::string::npos) return false;
    out = line.substr(a + pat.size(), b - a - pat.size());
    return true;
}

bool json_number(const std::string &line, const char *field, unsigned long long &out) {
    const std::string pat = std::string("\"") + field + "\": ";
    const size_t a = line.find(pat);
    if (a == std::string::npos) return false;
    char *end = nullptr;
    out = strtoull(line.c_str() + a + pat.size(), &end, 10);
    return end != line.c_str() + a + pat.size();
}

std::map<std::string, Tuned> read_tune_cache(const char *path) {
    std::map<std::string, Tuned> m;
    FILE *f = fopen(path, "r");
    if (!f) return m;
    char buf[1024];
    while (fgets(buf, sizeof(buf), f)) {
        const std::string line(buf);
        std::string key;
        unsigned long long th, tw, chunk, block, form, cap;
        if (!json_string(line, "key", key) || !json_number(line, "tile_rows", th) ||
            !json_number(line, "tile_cols", tw) || !json_number(line, "chunk", chunk) ||
            !json_number(line, "block", block) || !json_number(line, "form", form) ||
            !json_number(line, "pair_capacity", cap))
            continue;
        if (th < 1 || th > 256 || tw < 16 || tw > (unsigned long long)kMaxTileCells || th * tw > kMaxTileCells ||
            chunk < 64 || (block != 256 && block != 512 && block != 1024) || form > 2 || cap < 1)
            continue;
        Tuned t;
        t.plan.Th = (int)th;
        t.plan.Tw = (int)tw;
        t.plan.chunk = (int)chunk;
        t.plan.block = (int)block;
        t.plan.form = (int)form;
        t.plan.cap = 0;
        t.plan.counts = 1;
        t.plan.limit = 0;
        t.chunk = (int)chunk;
        t.cap = cap;
        m[key] = t;
    }
    fclose(f);
    return m;
}

void write_tune_cache(const char *path, const std::string &key, const Tuned &t) {
    std::map<std::string, Tuned> m = read_tune_cache(path);
    m[key] = t;
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = fopen(tmp.c_str(), "w");
    if (!f) return;  // the cache is an optimisation: a failed write is ignored
    fprintf(f, "{\"version\": 1, \"entries\": [\n");
    size_t i = 0;
    for (const auto &kv : m) {
        const Tuned &e = kv.second;
        fprintf(f,
                "{\"key\": \"%s\", \"tile_rows\": %d, \"tile_cols\": %d, \"chunk\": %d, \"block\": %d, "
                "\"form\": %d, \"pair_capacity\": %llu}%s\n",
                kv.first.c_str(), e.plan.Th, e.plan.Tw, e.chunk, e.plan.block, e.plan.form, e.cap,
                ++i < m.size() ? "," : "");
    }
    fprintf(f, "]}\n");
    const bool ok = fclose(f) == 0;
    if (ok) (void)rename(tmp.c_str(), path);
}

// Pair count of every (snapshot, view) image under `plan`: the front of each
// image (setup, count, scan, totals) into its own PlanOut slot, then one
// synchronisation.  Returns the counts in host_plan.
tess_status count_all(const tess_lattice *snaps, int n_snaps, const tess_view *views, int n_views, const Plan &plan,
                      hipStream_t s, Workspace &ws) {
    const int n_img = n_snaps * n_views;
    Sizes z;
    for (int i = 0; i < n_snaps; ++i)
        for (int v = 0; v < n_views; ++v) {
            Geometry g;
            tess_status st = make_geometry(snaps[i], &views[v], plan, g);
            if (st != TESS_OK) return st;
            z.add(g);
        }
    tess_status st = ensure_front(ws, z);
    if (st != TESS_OK) return st;
    TESS_HIP(ws.plan.ensure((size_t)n_img));
    if (ws.host_plan_cap < (size_t)n_img) {
        TESS_HIP(hipHostFree(ws.host_plan));
        ws.host_plan = nullptr;
        ws.host_plan_cap = 0;
        TESS_HIP(hipHostMalloc((void **)&ws.host_plan, sizeof(PlanOut) * (size_t)n_img, hipHostMallocDefault));
        ws.host_plan_cap = (size_t)n_img;
    }
    for (int i = 0; i < n_snaps; ++i)
        for (int v = 0; v < n_views; ++v) {
            Geometry g;
            st = make_geometry(snaps[i], &views[v], plan, g);
            if (st != TESS_OK) return st;
            st = enqueue_front(g, bufs_of(ws), ws.plan.p + i * n_views + v, ~0ull, nullptr, s);
            if (st != TESS_OK) return st;
        }
    TESS_HIP(hipMemcpyAsync(ws.host_plan, ws.plan.p, sizeof(PlanOut) * (size_t)n_img, hipMemcpyDeviceToHost, s));
    TESS_HIP(hipStreamSynchronize(s));
    return TESS_OK;
}

// The batch's tuning, done once per shape: the tiling (tune's, or the
// fastest candidate, timed on the image with the most pairs) and the pair
// capacity (tune's, or the largest count over all images under that tiling,
// with a small margin, so that no image of these snapshots overflows).
tess_status tune_batch(const tess_lattice *snaps, int n_snaps, const tess_view *views, int n_views,
                       const tess_tune *tune, float *scratch_image, hipStream_t s, Workspace &ws, Tuned &out) {
    const int n_img = n_snaps * n_views;
    Plan plan = choose_plan(&views[0], tune);
    if (!tune || (!tune->tile_rows && !tune->tile_cols)) {
        tess_status st = count_all(snaps, n_snaps, views, n_views, plan, s, ws);
        if (st != TESS_OK) return st;
        int heavy = 0;
        for (int k = 1; k < n_img; ++k)
            if (ws.host_plan[k].total_pairs > ws.host_plan[heavy].total_pairs) heavy = k;
        const tess_lattice hs = snaps[heavy / n_views];
        const tess_view *hv = &views[heavy % n_views];
        const int W = views[0].width;
        std::vector<Plan> cands;
        for (int Tw : {std::min(W, 1024), std::min(W, 512), std::min(W, 256)}) {
            for (int Th : {8, 16, 32, 64}) {
                if ((int64_t)Th * Tw > kMaxTileCells || (int64_t)Th * Tw < 2048) continue;
                bool dup = false;
                for (const Plan &c : cands) dup |= (c.Th == Th && c.Tw == Tw);
                if (dup) continue;
                Plan p = plan;
                p.Th = Th;
                p.Tw = Tw;
                p.cap = 0;
                cands.push_back(p);
            }
        }
        if (!cands.empty()) {
            float best_ms = 0;
            Plan best = cands[0];
            for (size_t c = 0; c < cands.size(); ++c) {
                float ms = 0;
                for (int rep = 0; rep < 2; ++rep) {  // the first call sizes the pair buffer
                    tess_stats st;
                    std::memset(&st, 0, sizeof(st));
                    tess_status rc = project_impl(hs, hv, cands[c], scratch_image, &st, s, ws);
                    if (rc != TESS_OK) return rc;
                    ms = st.ms;
                }
                if (c == 0 || ms < best_ms) {
                    best_ms = ms;
                    best = cands[c];
                }
            }
            best.cap = plan.cap;
            plan = best;
        }
    }
    unsigned long long most = 0;
    if (!plan.cap || !plan.chunk) {
        tess_status st = count_all(snaps, n_snaps, views, n_views, plan, s, ws);
        if (st != TESS_OK) return st;
        for (int k = 0; k < n_img; ++k) most = std::max<unsigned long long>(most, ws.host_plan[k].total_pairs);
    }
    out.plan = plan;
    out.chunk = plan.chunk ? plan.chunk : auto_chunk(most);
    out.cap = plan.cap ? plan.cap : most + most / 16 + 4096;
    return TESS_OK;
}

std::string graph_key(const tess_lattice *snaps, int n_snaps, const tess_view *views, int n_views, float *images,
                      const Tuned &t, int64_t own_cap, const Workspace &ws) {
    std::string k;
    auto put = [&](const void *p, size_t n) { k.append((const char *)p, n); };
    for (int i = 0; i < n_snaps; ++i) {
        put(&snaps[i]->desc, sizeof(tess_build_desc));
        put(&snaps[i]->x, sizeof(void *));
        put(&snaps[i]->y, sizeof(void *));
        put(&snaps[i]->z, sizeof(void *));
    }
    put(views, sizeof(tess_view) * (size_t)n_views);
    put(&images, sizeof(images));
    put(&t, sizeof(t));
    put(&own_cap, sizeof(own_cap));
    const void *bufs[] = {ws.head.p, ws.coef.p, ws.ecoef.p, ws.kinks.p, ws.sil.p, ws.spill.p, ws.counts.p, ws.base.p,
                          ws.scan.p, ws.tile_items.p, ws.items.p, ws.pairs.p, ws.acc.p, ws.plan.p, ws.counters.p,
                          ws.overflow.p};
    put(bufs, sizeof(bufs));
    return k;
}

tess_status project_batch_impl(const tess_lattice *snaps, int n_snaps, const tess_view *views, int n_views,
                               const tess_tune *tune, float *images, tess_stats *stats, hipStream_t s,
                               Workspace &ws) {
    const size_t img = (size_t)views[0].width * views[0].height;
    const int n_img = n_snaps * n_views;
    const std::string key = shape_key(snaps[0], &views[0], n_snaps, n_views, tune);
    const std::string count_key = "batch|" + key;
    // raster parameters and capacity: this process's, the cache file's, or tuned now
    Tuned t;
    bool have = false;
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        auto it = g_tuned.find(key);
        if (it != g_tuned.end()) {
            t = it->second;
            have = true;
        } else if (const char *path = tune_cache_path()) {
            std::map<std::string, Tuned> m = read_tune_cache(path);
            auto jt = m.find(key);
            if (jt != m.end()) {
                t = jt->second;
                g_tuned[key] = t;
                have = true;
            }
        }
    }
    if (!have) {
        tess_status rc = tune_batch(snaps, n_snaps, views, n_views, tune, images, s, ws, t);
        if (rc != TESS_OK) return rc;
        std::lock_guard<std::mutex> lock(g_tune_mu);
        g_tuned[key] = t;
        if (const char *path = tune_cache_path()) write_tune_cache(path, key, t);
    }
    // this call's workspace limit, whatever tuning the shape got
    t.plan.limit = choose_plan(&views[0], tune).limit;
    // counts of an earlier call that overflowed raise the capacity
    take_feedback(ws, s);
    {
        auto it = ws.learned.find(count_key);
        if (it != ws.learned.end() && it->second > t.cap && !t.plan.cap) {
            t.cap = capacity_for(it->second);
            std::lock_guard<std::mutex> lock(g_tune_mu);
            g_tuned[key] = t;
        }
    }
    // buffers for the largest image of the batch (forms and sizes may differ
    // between images), then the graph; edge-form images store the payloads of
    // as many tetrahedra with own records as the batch was seen to need
    int64_t own_cap = -1;
    {
        Geometry g0;
        tess_status st = make_geometry(snaps[0], &views[0], t.plan, g0);
        if (st != TESS_OK) return st;
        own_cap = own_capacity(ws, g0, count_key, t.plan);
    }
    Sizes z;
    for (int i = 0; i < n_snaps; ++i)
        for (int v = 0; v < n_views; ++v) {
            Geometry g;
            tess_status st = make_geometry(snaps[i], &views[v], t.plan, g, own_cap);
            if (st != TESS_OK) return st;
            z.add(g);
        }
    tess_status st = check_limit(ws, t.plan, z, t.chunk, t.cap, (size_t)n_img);
    if (st != TESS_OK) return st;
    st = ensure_front(ws, z);
    if (st != TESS_OK) return st;
    st = ensure_back(ws, z.ntiles, t.chunk, t.cap);
    if (st != TESS_OK) return st;
    TESS_HIP(ws.plan.ensure((size_t)n_img));
    if (ws.host_plan_cap < (size_t)n_img) {
        TESS_HIP(hipHostFree(ws.host_plan));
        ws.host_plan = nullptr;
        ws.host_plan_cap = 0;
        TESS_HIP(hipHostMalloc((void **)&ws.host_plan, sizeof(PlanOut) * (size_t)n_img, hipHostMallocDefault));
        ws.host_plan_cap = (size_t)n_img;
    }
    const std::string gkey = graph_key(snaps, n_snaps, views, n_views, images, t, own_cap, ws);
    if (!ws.graph || ws.graph_key != gkey) {
        if (ws.graph) {
            TESS_HIP(hipGraphExecDestroy(ws.graph));
            ws.graph = nullptr;
        }
        hipStream_t c = ws.capture;
        TESS_HIP(hipStreamBeginCapture(c, hipStreamCaptureModeThreadLocal));
        auto record = [&]() -> tess_status {
            TESS_HIP(launch_zero((double *)ws.counters.p, sizeof(DevCounters) / sizeof(double), c));
            for (int i = 0; i < n_snaps; ++i)
                for (int v = 0; v < n_views; ++v) {
                    const int k = i * n_views + v;
                    Geometry g;
                    tess_status r = make_geometry(snaps[i], &views[v], t.plan, g, own_cap);
                    if (r != TESS_OK) return r;
                    r = enqueue_front(g, bufs_of(ws), ws.plan.p + k, t.cap, nullptr, c);
                    if (r != TESS_OK) return r;
                    // the graph serves calls with and without stats: it counts
                    r = enqueue_back(g, t.plan, t.chunk, t.cap, true, bufs_of(ws), ws.plan.p + k, images + (size_t)k * img,
                                     c, nullptr, nullptr);
                    if (r != TESS_OK) return r;
                }
            return TESS_OK;
        };
        const tess_status cst = record();
        hipGraph_t graph = nullptr;
        const hipError_t end = hipStreamEndCapture(c, &graph);
        if (cst != TESS_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return cst;
        }
        if (end != hipSuccess) return fail(TESS_EHIP, "batch graph capture: %s", hipGetErrorString(end));
        const hipError_t inst = hipGraphInstantiate(&ws.graph, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (inst != hipSuccess) {
            ws.graph = nullptr;
            return fail(TESS_EHIP, "batch graph instantiation: %s", hipGetErrorString(inst));
        }
        ws.graph_key = gkey;
    }
    if (stats) TESS_HIP(hipEventRecord(ws.ev[0], s));
    TESS_HIP(hipGraphLaunch(ws.graph, s));
    if (!stats) return give_feedback(ws, ws.plan.p, n_img, count_key, s);
    TESS_HIP(hipEventRecord(ws.ev[4], s));
    TESS_HIP(hipMemcpyAsync(ws.host_plan, ws.plan.p, sizeof(PlanOut) * (size_t)n_img, hipMemcpyDeviceToHost, s));
    TESS_HIP(hipMemcpyAsync(ws.host_counters, ws.counters.p, sizeof(DevCounters), hipMemcpyDeviceToHost, s));
    TESS_HIP(hipStreamSynchronize(s));
    tess_stats acc;
    std::memset(&acc, 0, sizeof(acc));
    float ms = 0;
    TESS_HIP(hipEventElapsedTime(&ms, ws.ev[0], ws.ev[4]));
    fill_stats(&acc, *ws.host_counters, t.plan, t.chunk);
    acc.ms = ms;
    unsigned long long most = 0, own = 0;
    for (int k = 0; k < n_img; ++k) {
        const PlanOut &P = ws.host_plan[k];
        acc.bin_pairs += P.total_pairs;
        acc.max_bin = std::max<uint32_t>(acc.max_bin, (uint32_t)std::min<unsigned long long>(P.max_bin, 0xffffffffull));
        acc.work_items += (uint32_t)P.n_items;
        // (P.own is 0 for images not in the edge form)
        acc.overflow += P.total_pairs > t.cap || (own_cap >= 0 && P.own > (unsigned long long)own_cap) ? 1u : 0u;
        acc.own_records += (uint32_t)std::min<unsigned long long>(P.own, 0xffffffffull);
        most = std::max<unsigned long long>(most, P.total_pairs);
        own = std::max<unsigned long long>(own, P.own);
    }
    unsigned long long &m = ws.learned[count_key];
    m = std::max(m, most);
    if (own) {
        unsigned long long &o = ws.learned_own[count_key];
        o = std::max(o, own);
    }
    *stats = acc;
    return TESS_OK;
}
}  // namespace

extern "C" tess_status tess_project(tess_lattice L, const tess_view *v, const tess_tune *tune,
                                    float *image, tess_stats *stats, void *stream) {
    tess_status st = check_project_args(L, v, tune, image);
    if (st != TESS_OK) return st;
    if (stats) std::memset(stats, 0, sizeof(*stats));
    hipStream_t s = (hipStream_t)stream;
    Workspace *ws = nullptr;
    st = lock_workspace(L, s, &ws);
    if (st != TESS_OK) return st;
    std::lock_guard<std::mutex> lock(ws->mu);
    st = project_impl(L, v, choose_plan(v, tune), image, stats, s, *ws);
    return st == TESS_OK ? ok() : st;
}

// ------------------------------------------- allocation-free projection
namespace {
// Hands out 256-byte aligned pieces of the scratch, front to back.
struct Carve {
    unsigned char *base;
    size_t off = 0;
    template <typename T>
    T *take(size_t n) {
        off = (off + 255) & ~(size_t)255;
        T *p = reinterpret_cast<T *>(base + off);
        off += n * sizeof(T);
        return p;
    }
};
}  // namespace

extern "C" tess_status tess_project_noalloc(tess_lattice L, const tess_view *v, const tess_tune *tune,
                                            float *image, void *stream) {
    tess_status st = check_project_args(L, v, tune, image);
    if (st != TESS_OK) return st;
    int dev = 0;
    TESS_HIP(hipGetDevice(&dev));
    if (dev != L->device) return fail(TESS_EINVAL, "lattice lives on device %d, current device is %d", L->device, dev);
    hipStream_t s = (hipStream_t)stream;
    const Plan plan = choose_plan(v, tune);
    Geometry g;
    st = make_geometry(L, v, plan, g);
    if (st != TESS_OK) return st;
    void *sp = nullptr;
    TESS_HIP(scratch_buffer(&sp));
    // what tess_project's workspace holds for this image, then the pair list
    // (and its work items) in all the room that is left
    Carve c{static_cast<unsigned char *>(sp)};
    Bufs b;
    b.head = c.take<RecHead>((size_t)g.ntet);
    b.coef = c.take<Payload>((size_t)g.stored);
    const int64_t nvert = (int64_t)g.lp.d[0] * g.lp.d[1] * g.lp.d[2];
    b.ecoef = g.vp.edges ? c.take<EdgePayload>((size_t)(g.ntet - g.stored)) : nullptr;
    b.kinks = g.vp.edges ? c.take<double>((size_t)(36 * nvert)) : nullptr;
    b.sil = g.vp.edges ? c.take<uint8_t>((size_t)(36 * nvert)) : nullptr;
    b.spill = g.vp.edges ? c.take<uint32_t>((size_t)g.spill) : nullptr;
    b.counts = c.take<uint32_t>((size_t)g.nmat);
    b.base = c.take<uint64_t>((size_t)g.nmat);
    b.scan = c.take<uint64_t>(scan_scratch_elems(g.nmat));
    b.tile_items = c.take<uint32_t>((size_t)g.ntiles + 1);
    b.acc = c.take<double>((size_t)g.npix);
    PlanOut *slot = c.take<PlanOut>(1);
    b.counters = c.take<DevCounters>(1);
    const int chunk = plan.chunk ? plan.chunk : 1024;
    const size_t fixed = (c.off + 255) & ~(size_t)255;
    const size_t need = fixed + 512 + 16 * ((size_t)g.ntiles + 1) + 4 * 1024;
    if (need > kScratchBytes)
        return fail(TESS_ECAPACITY,
                    "this lattice and view need %.1f MiB of scratch; the allocation-free projection has %.0f MiB "
                    "(use tess_project)", need / 1048576.0, kScratchBytes / 1048576.0);
    // room for cap pairs (4 B) and cap / chunk + ntiles work items (16 B)
    const size_t room = kScratchBytes - fixed - 512 - 16 * ((size_t)g.ntiles + 1);
    unsigned long long cap = (unsigned long long)(room / (4.0 + 16.0 / chunk));
    if (plan.cap && plan.cap < cap) cap = plan.cap;
    b.items = c.take<WorkItem>((size_t)max_items_for(g.ntiles, chunk, cap));
    b.pairs = c.take<uint32_t>((size_t)cap);
    if (c.off > kScratchBytes) return fail(TESS_ECAPACITY, "scratch layout overflow");  // not reached
    TESS_HIP(launch_zero((double *)b.counters, sizeof(DevCounters) / sizeof(double), s));
    st = enqueue_setup(g, b, slot, s);
    if (st != TESS_OK) return st;
    TESS_HIP(launch_count(b.head, g.ntet, g.B, b.counts, s));
    TESS_HIP(launch_scan(b.counts, b.base, g.nmat, b.scan, s));
    TESS_HIP(launch_totals(b.counts, b.base, g.B, cap, slot, nullptr, s));
    st = enqueue_back(g, plan, chunk, cap, false, b, slot, image, s, nullptr, nullptr);
    return st == TESS_OK ? ok() : st;
}

extern "C" tess_status tess_project_batch(const tess_lattice *snaps, int32_t n_snaps,
                                          const tess_view *views, int32_t n_views,
                                          const tess_tune *tune, float *images, tess_stats *stats,
                                          void *stream) {
    if (!snaps || !views || !images) return fail(TESS_EINVAL, "NULL argument");
    if (n_snaps < 1 || n_views < 1) return fail(TESS_EINVAL, "need at least one snapshot and one view");
    for (int32_t s = 0; s < n_snaps; ++s) {
        if (!snaps[s]) return fail(TESS_EINVAL, "snapshot %d is NULL", s);
        for (int a = 0; a < 3; ++a)
            if (snaps[s]->desc.dims[a] != snaps[0]->desc.dims[a])
                return fail(TESS_EINVAL, "snapshot %d has different dims", s);
        if (snaps[s]->desc.periodic != snaps[0]->desc.periodic)
            return fail(TESS_EINVAL, "snapshot %d differs in periodicity", s);
        if (snaps[s]->device != snaps[0]->device)
            return fail(TESS_EINVAL, "snapshot %d lives on another device", s);
    }
    for (int32_t v = 0; v < n_views; ++v) {
        if (views[v].width != views[0].width || views[v].height != views[0].height)
            return fail(TESS_EINVAL, "view %d has a different image size", v);
        for (int32_t s = 0; s < n_snaps; ++s) {
            tess_status st = check_project_args(snaps[s], &views[v], tune, images);
            if (st != TESS_OK) return st;
        }
    }
    if (stats) std::memset(stats, 0, sizeof(*stats));
    hipStream_t s = (hipStream_t)stream;
    Workspace *ws = nullptr;
    tess_status st = lock_workspace(snaps[0], s, &ws);
    if (st != TESS_OK) return st;
    std::lock_guard<std::mutex> lock(ws->mu);
    st = project_batch_impl(snaps, n_snaps, views, n_views, tune, images, stats, s, *ws);
    return st == TESS_OK ? ok() : st;
}

extern "C" const char *tess_last_error(void) { return g_error.c_str(); }

extern "C" int32_t tess_version(void) { return 100; }

extern "C" uint64_t tess_struct_size(int32_t which) {
    switch (which) {
        case 0: return sizeof(tess_build_desc);
        case 1: return sizeof(tess_view);
        case 2: return sizeof(tess_tune);
        case 3: return sizeof(tess_stats);
        case 4: return sizeof(tess_refine_desc);
        default: return 0;
    }
}
