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
    // batch graph (captured on `capture`, replayed on the caller's stream)
    hipStream_t capture = nullptr;
    hipGraphExec_t graph = nullptr;
    std::string graph_key;
    std::mutex mu;
};

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

extern "C" void tess_free(tess_lattice L) {
    if (!L) return;
    if (L->owned) (void)hipFree(L->owned);
    delete L;
}

// ------------------------------------------------------------ projection
namespace {
void make_params(const tess_lattice_s *L, const tess_view *v, LatticeParams &lp, ViewParams &vp) {
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
    // Plain pyramids take the edge form when a lattice cell spans at least
    // 6 pixels: its cost per lattice vertex (the edge records) then buys a
    // larger saving in the raster, whose work grows with the rows each
    // tetrahedron covers (measured: 2 pixels per cell, 512 rotated 512^2
    // windows on 128^3, favour the per-tetrahedron form; 8 pixels per cell
    // and more favour the edge form at every size tried).  TESS_PER_TETRAHEDRON=1 forces the
    // per-tetrahedron form and =0 the edge form (the two give the same image
    // up to rounding).
    const double cell_px = std::cbrt(d.box[0] * d.box[1] * d.box[2] / (double)lp.ncubes) *
                           std::sqrt(vp.inv_du * vp.inv_dv);
    const char *per_tet = getenv("TESS_PER_TETRAHEDRON");
    const bool force_tet = per_tet && per_tet[0] == '1', force_edges = per_tet && per_tet[0] == '0';
    vp.edges = (view_form(vp) == kFormPyramid && !force_tet && (force_edges || cell_px >= 6.0)) ? 1 : 0;
    vp.kinks = nullptr;
    vp.sil = nullptr;
}

struct Plan {
    int Th, Tw, chunk, block;  // chunk 0: from the pair count
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
};

tess_status make_geometry(const tess_lattice_s *L, const tess_view *v, const Plan &plan, Geometry &g) {
    make_params(L, v, g.lp, g.vp);
    // records: the tetrahedra, then (edge form) seven edges per lattice vertex;
    // the edge form only while all ids fit in 32 bits
    const int64_t nvert = (int64_t)g.lp.d[0] * g.lp.d[1] * g.lp.d[2];
    if (g.vp.edges && 6 * g.lp.ncubes + 7 * nvert >= (int64_t)0xffffffff) g.vp.edges = 0;
    g.ntet = 6 * g.lp.ncubes + (g.vp.edges ? 7 * nvert : 0);
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
    B.first_edge = (uint32_t)(6 * g.lp.ncubes);
    B.seam = g.vp.edges && v->wrap ? 1 : 0;
    g.nmat = g.ntiles * B.nseg;
    g.npix = (int64_t)B.W * B.H;
    return TESS_OK;
}

tess_status ensure_front(Workspace &ws, const Geometry &g) {
    TESS_HIP(ws.head.ensure((size_t)g.ntet));
    TESS_HIP(ws.coef.ensure((size_t)(6 * g.lp.ncubes)));
    if (g.vp.edges) TESS_HIP(ws.ecoef.ensure((size_t)(g.ntet - 6 * g.lp.ncubes)));
    if (g.vp.edges) {
        const size_t slots = (size_t)36 * (size_t)g.lp.d[0] * (size_t)g.lp.d[1] * (size_t)g.lp.d[2];
        TESS_HIP(ws.kinks.ensure(slots));
        TESS_HIP(ws.sil.ensure(slots));
    }
    TESS_HIP(ws.counts.ensure((size_t)g.nmat));
    TESS_HIP(ws.base.ensure((size_t)g.nmat));
    TESS_HIP(ws.scan.ensure(scan_scratch_elems(g.nmat)));
    TESS_HIP(ws.tile_items.ensure((size_t)g.ntiles + 1));
    TESS_HIP(ws.acc.ensure((size_t)g.npix));
    TESS_HIP(ws.counters.ensure(1));
    TESS_HIP(ws.overflow.ensure(1));
    return TESS_OK;
}

unsigned long long max_items_for(const Geometry &g, int chunk, unsigned long long cap) {
    return cap / (unsigned long long)chunk + (unsigned long long)g.ntiles;
}

tess_status ensure_back(Workspace &ws, const Geometry &g, int chunk, unsigned long long cap) {
    TESS_HIP(ws.items.ensure((size_t)std::max<unsigned long long>(max_items_for(g, chunk, cap), 1)));
    TESS_HIP(ws.pairs.ensure((size_t)std::max<unsigned long long>(cap, 1)));
    return TESS_OK;
}

// Setup, count, scan and totals of one image (no host synchronisation).
// Setup of one image; for q = 1 first the integral of q into slot->qsum.
tess_status enqueue_setup(const Geometry &g, Workspace &ws, PlanOut *slot, hipStream_t s) {
    ViewParams vp = g.vp;
    if (vp.qpow == 0 && !vp.slab && !vp.splat && !vp.persp) {
        TESS_HIP(launch_zero(&slot->qsum, 1, s));
        TESS_HIP(launch_qsum(g.lp, vp, &slot->qsum, s));
        vp.qsum = &slot->qsum;
    }
    vp.kinks = ws.kinks.p;
    vp.sil = ws.sil.p;
    TESS_HIP(launch_setup(g.lp, vp, ws.head.p, ws.coef.p, ws.counters.p, s));
    if (vp.edges) TESS_HIP(launch_edges(g.lp, vp, ws.head.p, ws.ecoef.p, s));
    return TESS_OK;
}

tess_status enqueue_front(const Geometry &g, Workspace &ws, PlanOut *slot, unsigned long long cap,
                          unsigned int *overflow, hipStream_t s) {
    tess_status st = enqueue_setup(g, ws, slot, s);
    if (st != TESS_OK) return st;
    TESS_HIP(launch_count(ws.head.p, g.ntet, g.B, ws.counts.p, s));
    TESS_HIP(launch_scan(ws.counts.p, ws.base.p, g.nmat, ws.scan.p, s));
    TESS_HIP(launch_totals(ws.counts.p, ws.base.p, g.B, cap, slot, overflow, s));
    return TESS_OK;
}

// Work items, scatter, raster and finalize of one image into `image`, for at
// most `cap` pairs (the buffers hold that many).
tess_status enqueue_back(const Geometry &g, const Plan &plan, int chunk, unsigned long long cap,
                         Workspace &ws, PlanOut *slot, float *image, hipStream_t s, hipEvent_t after_bin,
                         hipEvent_t after_raster) {
    TESS_HIP(launch_plan(ws.counts.p, ws.base.p, g.B, chunk, cap, ws.tile_items.p, slot, s));
    TESS_HIP(launch_items(ws.base.p, ws.tile_items.p, g.B, chunk, slot, ws.items.p, s));
    TESS_HIP(launch_scatter(ws.head.p, g.ntet, g.B, ws.base.p, ws.pairs.p, cap, s));
    TESS_HIP(launch_zero(ws.acc.p, g.npix, s));
    if (after_bin) TESS_HIP(hipEventRecord(after_bin, s));
    TESS_HIP(launch_raster(ws.head.p, ws.coef.p, ws.ecoef.p, ws.pairs.p, ws.items.p, max_items_for(g, chunk, cap), slot,
                           g.B, plan.block, ws.acc.p, ws.counters.p, s));
    if (after_raster) TESS_HIP(hipEventRecord(after_raster, s));
    TESS_HIP(launch_finalize(ws.acc.p, g.B, image, s));
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

// One image, synchronising once to size the pair buffer from its own count.
tess_status project_impl(const tess_lattice_s *L, const tess_view *v, const Plan &plan, float *image,
                         tess_stats *stats, hipStream_t s, Workspace &ws) {
    Geometry g;
    tess_status st = make_geometry(L, v, plan, g);
    if (st != TESS_OK) return st;
    st = ensure_front(ws, g);
    if (st != TESS_OK) return st;
    TESS_HIP(ws.plan.ensure(1));
    if (stats) TESS_HIP(hipEventRecord(ws.ev[0], s));
    TESS_HIP(launch_zero((double *)ws.counters.p, sizeof(DevCounters) / sizeof(double), s));
    st = enqueue_setup(g, ws, ws.plan.p, s);
    if (st != TESS_OK) return st;
    if (stats) TESS_HIP(hipEventRecord(ws.ev[1], s));
    TESS_HIP(launch_count(ws.head.p, g.ntet, g.B, ws.counts.p, s));
    TESS_HIP(launch_scan(ws.counts.p, ws.base.p, g.nmat, ws.scan.p, s));
    TESS_HIP(launch_totals(ws.counts.p, ws.base.p, g.B, ~0ull, ws.plan.p, nullptr, s));
    TESS_HIP(hipMemcpyAsync(ws.host_plan, ws.plan.p, sizeof(PlanOut), hipMemcpyDeviceToHost, s));
    TESS_HIP(hipStreamSynchronize(s));
    const unsigned long long total = ws.host_plan->total_pairs;
    const int chunk = plan.chunk ? plan.chunk : auto_chunk(total);
    st = ensure_back(ws, g, chunk, total);
    if (st != TESS_OK) return st;
    st = enqueue_back(g, plan, chunk, total, ws, ws.plan.p, image, s, stats ? ws.ev[2] : nullptr,
                      stats ? ws.ev[3] : nullptr);
    if (st != TESS_OK) return st;
    if (stats) {
        TESS_HIP(hipEventRecord(ws.ev[4], s));
        TESS_HIP(hipMemcpyAsync(ws.host_counters, ws.counters.p, sizeof(DevCounters),
                                hipMemcpyDeviceToHost, s));
        TESS_HIP(hipMemcpyAsync(ws.host_plan, ws.plan.p, sizeof(PlanOut), hipMemcpyDeviceToHost, s));
        TESS_HIP(hipStreamSynchronize(s));
        float ms = 0, t_setup = 0, t_bin = 0, t_raster = 0, t_fin = 0;
        TESS_HIP(hipEventElapsedTime(&ms, ws.ev[0], ws.ev[4]));
        TESS_HIP(hipEventElapsedTime(&t_setup, ws.ev[0], ws.ev[1]));
        TESS_HIP(hipEventElapsedTime(&t_bin, ws.ev[1], ws.ev[2]));
        TESS_HIP(hipEventElapsedTime(&t_raster, ws.ev[2], ws.ev[3]));
        TESS_HIP(hipEventElapsedTime(&t_fin, ws.ev[3], ws.ev[4]));
        const PlanOut &P = *ws.host_plan;
        fill_stats(stats, *ws.host_counters, plan, chunk);
        stats->bin_pairs = P.total_pairs;
        stats->max_bin = (uint32_t)std::min<unsigned long long>(P.max_bin, 0xffffffffull);
        stats->work_items = (uint32_t)P.n_items;
        stats->ms = ms;
        stats->setup_ms = t_setup;
        stats->bin_ms = t_bin;
        stats->raster_ms = t_raster;
        stats->finalize_ms = t_fin;
    }
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
// later calls with the same lattice and image shape.
struct Tuned {
    Plan plan;
    int chunk;
    unsigned long long cap;
};
std::mutex g_tune_mu;
std::map<std::string, Tuned> g_tuned;

std::string shape_key(const tess_lattice_s *L, const tess_view *v, int n_snaps, int n_views) {
    char buf[256];
    snprintf(buf, sizeof(buf), "%d:%d:%d:%d|%dx%d:%d|%d:%d", L->desc.dims[0], L->desc.dims[1], L->desc.dims[2],
             L->desc.periodic, v->width, v->height, v->wrap, n_snaps, n_views);
    return buf;
}

// Times one image under each candidate tiling (synchronous calls) and keeps
// the fastest; the pair capacity is 1.5 times the largest count seen over the
// snapshots' first views.
tess_status autotune(const tess_lattice *snaps, int n_snaps, const tess_view *views, float *scratch_image,
                     hipStream_t s, Workspace &ws, Tuned &out) {
    Plan base = choose_plan(&views[0], nullptr);
    unsigned long long most = 0;
    int heavy = 0;
    for (int i = 0; i < n_snaps; ++i) {
        tess_stats st;
        std::memset(&st, 0, sizeof(st));
        tess_status rc = project_impl(snaps[i], &views[0], base, scratch_image, &st, s, ws);
        if (rc != TESS_OK) return rc;
        if (st.bin_pairs >= most) {
            most = st.bin_pairs;
            heavy = i;
        }
    }
    const int W = views[0].width;
    std::vector<Plan> cands;
    for (int Tw : {std::min(W, 1024), std::min(W, 512), std::min(W, 256)}) {
        for (int Th : {8, 16, 32, 64}) {
            if ((int64_t)Th * Tw > kMaxTileCells || (int64_t)Th * Tw < 2048) continue;
            bool dup = false;
            for (const Plan &c : cands) dup |= (c.Th == Th && c.Tw == Tw);
            if (dup) continue;
            Plan p = base;
            p.Th = Th;
            p.Tw = Tw;
            cands.push_back(p);
        }
    }
    if (cands.empty()) cands.push_back(base);
    float best_ms = 0;
    Plan best = cands[0];
    for (const Plan &p : cands) {
        float ms = 0;
        for (int rep = 0; rep < 2; ++rep) {
            tess_stats st;
            std::memset(&st, 0, sizeof(st));
            tess_status rc = project_impl(snaps[heavy], &views[0], p, scratch_image, &st, s, ws);
            if (rc != TESS_OK) return rc;
            ms = st.ms;
        }
        if (&p == &cands[0] || ms < best_ms) {
            best_ms = ms;
            best = p;
        }
    }
    out.plan = best;
    out.chunk = auto_chunk(most);
    out.cap = most + most / 2 + 4096;
    return TESS_OK;
}

std::string graph_key(const tess_lattice *snaps, int n_snaps, const tess_view *views, int n_views, float *images,
                      const Tuned &t, const Workspace &ws) {
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
    const void *bufs[] = {ws.head.p, ws.coef.p, ws.ecoef.p, ws.kinks.p, ws.sil.p, ws.counts.p, ws.base.p, ws.scan.p, ws.tile_items.p,
                          ws.items.p, ws.pairs.p, ws.acc.p, ws.plan.p, ws.counters.p, ws.overflow.p};
    put(bufs, sizeof(bufs));
    const char *per_tet = getenv("TESS_PER_TETRAHEDRON");
    const char form = per_tet ? per_tet[0] : 'x';  // the form switch
    put(&form, 1);
    return k;
}

tess_status project_batch_impl(const tess_lattice *snaps, int n_snaps, const tess_view *views, int n_views,
                               const tess_tune *tune, float *images, tess_stats *stats, hipStream_t s,
                               Workspace &ws) {
    const size_t img = (size_t)views[0].width * views[0].height;
    const int n_img = n_snaps * n_views;
    // raster parameters and capacity, sized once per batch shape and tune
    Tuned t;
    std::string key = shape_key(snaps[0], &views[0], n_snaps, n_views);
    if (tune) {
        char buf[96];
        snprintf(buf, sizeof(buf), "|tune %d %d %d %d", tune->tile_rows, tune->tile_cols, tune->chunk, tune->block);
        key += buf;
    }
    bool have = false;
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        auto it = g_tuned.find(key);
        if (it != g_tuned.end()) {
            t = it->second;
            have = true;
        }
    }
    if (!have) {
        if (tune) {
            t.plan = choose_plan(&views[0], tune);
            unsigned long long most = 0;
            for (int i = 0; i < n_snaps; ++i) {
                tess_stats st;
                std::memset(&st, 0, sizeof(st));
                tess_status rc = project_impl(snaps[i], &views[0], t.plan, images, &st, s, ws);
                if (rc != TESS_OK) return rc;
                most = std::max<unsigned long long>(most, st.bin_pairs);
            }
            t.chunk = t.plan.chunk ? t.plan.chunk : auto_chunk(most);
            t.cap = most + most / 2 + 4096;
        } else {
            tess_status rc = autotune(snaps, n_snaps, views, images, s, ws, t);
            if (rc != TESS_OK) return rc;
        }
        std::lock_guard<std::mutex> lock(g_tune_mu);
        g_tuned[key] = t;
    }
    // buffers for the largest image of the batch, then the graph
    Geometry g0;
    tess_status st = make_geometry(snaps[0], &views[0], t.plan, g0);
    if (st != TESS_OK) return st;
    st = ensure_front(ws, g0);
    if (st != TESS_OK) return st;
    st = ensure_back(ws, g0, t.chunk, t.cap);
    if (st != TESS_OK) return st;
    TESS_HIP(ws.plan.ensure((size_t)n_img));
    if (ws.host_plan_cap < (size_t)n_img) {
        TESS_HIP(hipHostFree(ws.host_plan));
        ws.host_plan = nullptr;
        TESS_HIP(hipHostMalloc((void **)&ws.host_plan, sizeof(PlanOut) * (size_t)n_img, hipHostMallocDefault));
        ws.host_plan_cap = (size_t)n_img;
    }
    const std::string gkey = graph_key(snaps, n_snaps, views, n_views, images, t, ws);
    if (!ws.graph || ws.graph_key != gkey) {
        if (ws.graph) {
            TESS_HIP(hipGraphExecDestroy(ws.graph));
            ws.graph = nullptr;
        }
        hipStream_t c = ws.capture;
        TESS_HIP(hipStreamBeginCapture(c, hipStreamCaptureModeThreadLocal));
        tess_status cst = TESS_OK;
        auto record = [&]() -> tess_status {
            TESS_HIP(launch_zero((double *)ws.counters.p, sizeof(DevCounters) / sizeof(double), c));
            TESS_HIP(launch_zero((double *)ws.overflow.p, 1, c));  // the buffer holds >= 64 words
            for (int i = 0; i < n_snaps; ++i)
                for (int v = 0; v < n_views; ++v) {
                    const int k = i * n_views + v;
                    Geometry g;
                    tess_status r = make_geometry(snaps[i], &views[v], t.plan, g);
                    if (r != TESS_OK) return r;
                    r = enqueue_front(g, ws, ws.plan.p + k, t.cap, ws.overflow.p, c);
                    if (r != TESS_OK) return r;
                    r = enqueue_back(g, t.plan, t.chunk, t.cap, ws, ws.plan.p + k, images + (size_t)k * img, c,
                                     nullptr, nullptr);
                    if (r != TESS_OK) return r;
                }
            return TESS_OK;
        };
        cst = record();
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
    if (stats) TESS_HIP(hipEventRecord(ws.ev[4], s));
    TESS_HIP(hipMemcpyAsync(ws.host_overflow, ws.overflow.p, sizeof(unsigned int), hipMemcpyDeviceToHost, s));
    TESS_HIP(hipMemcpyAsync(ws.host_plan, ws.plan.p, sizeof(PlanOut) * (size_t)n_img, hipMemcpyDeviceToHost, s));
    TESS_HIP(hipMemcpyAsync(ws.host_counters, ws.counters.p, sizeof(DevCounters), hipMemcpyDeviceToHost, s));
    TESS_HIP(hipStreamSynchronize(s));
    tess_stats acc;
    std::memset(&acc, 0, sizeof(acc));
    if (stats) {
        float ms = 0;
        TESS_HIP(hipEventElapsedTime(&ms, ws.ev[0], ws.ev[4]));
        fill_stats(&acc, *ws.host_counters, t.plan, t.chunk);
        acc.ms = ms;
        for (int k = 0; k < n_img; ++k) {
            acc.bin_pairs += ws.host_plan[k].total_pairs;
            acc.max_bin = std::max<uint32_t>(acc.max_bin, (uint32_t)std::min<unsigned long long>(
                                                              ws.host_plan[k].max_bin, 0xffffffffull));
            acc.work_items += (uint32_t)ws.host_plan[k].n_items;
        }
    }
    if (*ws.host_overflow) {
        // images whose pairs exceeded the capacity: redo them one by one
        std::vector<int> redo;
        for (int k = 0; k < n_img; ++k)
            if (ws.host_plan[k].total_pairs > t.cap) redo.push_back(k);
        for (int k : redo) {
            tess_stats one;
            std::memset(&one, 0, sizeof(one));
            const int i = k / n_views, v = k % n_views;
            tess_status rc = project_impl(snaps[i], &views[v], t.plan, images + (size_t)k * img,
                                          stats ? &one : nullptr, s, ws);
            if (rc != TESS_OK) return rc;
            if (stats) {
                // the graph's counters missed this image's raster
                acc.fragments += one.fragments;
                acc.spans += one.spans;
                acc.kinks += one.kinks;
                acc.work_items += one.work_items;
                acc.ms += one.ms;
            }
        }
        // the next call sizes for the largest count seen
        unsigned long long most = 0;
        for (int k = 0; k < n_img; ++k) most = std::max<unsigned long long>(most, ws.host_plan[k].total_pairs);
        {
            std::lock_guard<std::mutex> lock(g_tune_mu);
            auto it = g_tuned.find(key);
            if (it != g_tuned.end()) it->second.cap = most + most / 2 + 4096;
        }
    }
    if (stats) *stats = acc;
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
