// HIP kernels of the tessellation projector (gfx950).
//
// Pipeline of one projection (all on the caller's stream):
//   k_setup    one thread per lattice cube: gather the 8 corners (coalesced
//              SoA loads), unwrap them to the periodic image nearest corner 0,
//              cut the cube into the six tetrahedra of the connectivity table,
//              compute the volume determinant (Eq. Eqn:TetVolume; FP32, redone
//              in FP64 when flagged) and the tetrahedron's screen footprint
//              (FP64), stored as FP32 coefficients, or as FP64 ones in a side
//              array when FP32 evaluation would be ill-conditioned.
//   k_count    per segment of tetrahedra: tiles touched by each footprint
//   k_scan     exclusive scan of the (tile, segment) counts
//   k_plan     per-tile lists split into raster work items of <= chunk entries
//   k_scatter  stable scatter of tetrahedron ids into the tile lists
//   k_raster   per work item: every lane owns a strip of pixels of the tile and
//              accumulates rho * dl of the listed tetrahedra in registers
//              (FP32 terms summed in FP32 blocks folded into FP64; FP64 terms
//              for the flagged footprints)
//   k_finalize sums the work-item partials of each tile in order -> image
//
// The footprint.  Under orthographic projection, rho * dl of one tetrahedron
// (the per-tetrahedron term of Eq. Eqn:TetProjection with q = m/V) is a
// pyramid over the projected silhouette: it vanishes on the silhouette and is
// linear between the silhouette edges and the apex.  It therefore equals
//     max(0, min over silhouette edges (i,j) of G_ij(p)),
//     G_ij(p) = 6 m * cross(q_j - q_i, p - q_i) / (D_ijk * |D_ijl|),
// where q are the projected vertices, k and l the two other vertices and
// D_ijk = cross(q_j - q_i, q_k - q_i).  An edge is on the silhouette exactly
// when q_k and q_l lie on the same side of it.  (The front/back split of
// Eq. Eqn:TetSum is the same function written as exit depth minus entry
// depth; this form needs only the projected vertices, so it is free of the
// depth cancellation of that split and of the 1/V of near-flat tetrahedra.)
// A face seen edge-on (projected determinant exactly 0) bounds the footprint
// as a "wall": a half-plane test, with the half-open tie rule for pixel
// centres exactly on it.
#include "tess_tet.h"

#include <cfloat>
#include <climits>

namespace tess {


__device__ inline unsigned long long wave_sum(unsigned long long v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// One thread per lattice cube; writes the six records 6*cube .. 6*cube+5 and
// hands out FP64 coefficient slots (one atomic per wavefront and tetrahedron).
__global__ void __launch_bounds__(256) k_setup(LatticeParams L, ViewParams V,
                                               TetRec *__restrict__ rec,
                                               Coef64 *__restrict__ coef64, uint32_t coef64_cap,
                                               DevCounters *__restrict__ counters) {
    CubeCounts cnt;
    unsigned long long n_f64 = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t nloop = (L.ncubes + stride - 1) / stride;  // same trip count on every lane
    const int64_t first = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    for (int64_t it = 0; it < nloop; ++it) {
        const int64_t cube = first + it * stride;
        const bool live = cube < L.ncubes;
        TetRec r[6];
        Footprint fp[6];
        bool want64[6] = {false, false, false, false, false, false};
        if (live) setup_cube(L, V, cube, r, fp, want64, cnt);
#pragma unroll
        for (int t = 0; t < 6; ++t) {
            const unsigned long long mask = __ballot(want64[t]);
            if (mask) {
                unsigned long long base = 0;
                const int leader = __ffsll((long long)mask) - 1;
                if (lane == leader) base = atomicAdd(&counters->coef64_used, (unsigned long long)__popcll(mask));
                base = __shfl(base, leader, 64);
                if (want64[t]) {
                    const unsigned long long slot = base + __popcll(mask & ((1ull << lane) - 1ull));
                    r[t].h.flags |= REC_FP64;
                    ++n_f64;
                    if (slot < coef64_cap) {
                        r[t].h.slot = (uint32_t)slot;
                        Coef64 cf;
#pragma unroll
                        for (int g = 0; g < 12; ++g) cf.c[g] = fp[t].c[g];
                        coef64[slot] = cf;
                    }
                }
            }
            if (live) rec[6 * cube + t] = r[t];
        }
    }
    const unsigned long long n_tets = wave_sum(cnt.n_tets), n_zero = wave_sum(cnt.n_zero),
                             n_inv = wave_sum(cnt.n_inv), n_dets = wave_sum(cnt.n_dets),
                             n_deg = wave_sum(cnt.n_deg);
    n_f64 = wave_sum(n_f64);
    if (lane == 0) {
        if (n_tets) atomicAdd(&counters->tets, n_tets);
        if (n_zero) atomicAdd(&counters->zero_volume, n_zero);
        if (n_inv) atomicAdd(&counters->inverted, n_inv);
        if (n_dets) atomicAdd(&counters->fp64_dets, n_dets);
        if (n_f64) atomicAdd(&counters->fp64_tets, n_f64);
        if (n_deg) atomicAdd(&counters->degenerate, n_deg);
    }
}

hipError_t launch_setup(const LatticeParams &L, const ViewParams &V, TetRec *rec, Coef64 *coef64,
                        uint32_t coef64_cap, DevCounters *counters, hipStream_t stream) {
    const int64_t want = (L.ncubes + 255) / 256;
    const int blocks = (int)(want < 65536 ? (want > 0 ? want : 1) : 65536);
    hipLaunchKernelGGL(k_setup, dim3(blocks), dim3(256), 0, stream, L, V, rec, coef64, coef64_cap,
                       counters);
    return hipGetLastError();
}

// ---------------------------------------------------------------- binning
// One wavefront per segment of seg_len consecutive tetrahedra.  Tetrahedra
// are visited in id order; the lanes split one tetrahedron's candidate tiles,
// so every tile list ends up in id order (a stable counting sort on the tile
// key) whatever the scheduling.
template <bool SCATTER>
__global__ void __launch_bounds__(64) k_bin(const TetRec *__restrict__ rec, int64_t ntet,
                                            BinParams B, uint32_t *__restrict__ counts,
                                            const uint64_t *__restrict__ base,
                                            uint32_t *__restrict__ pairs,
                                            unsigned long long pair_cap) {
    extern __shared__ uint32_t lds_bins[];  // per tile: count, or next slot relative to tile start
    const int ntiles = B.ntx * B.nty;
    const int seg = blockIdx.x;
    const int lane = threadIdx.x;
    for (int t = lane; t < ntiles; t += 64) {
        if (SCATTER)
            lds_bins[t] = (uint32_t)(base[(int64_t)t * B.nseg + seg] - base[(int64_t)t * B.nseg]);
        else
            lds_bins[t] = 0;
    }
    __syncthreads();
    const int64_t t0 = (int64_t)seg * B.seg_len;
    const int64_t t1 = min(ntet, t0 + B.seg_len);
    for (int64_t id = t0; id < t1; ++id) {
        const TetRec r = rec[id];
        if (!(r.h.flags & REC_VALID)) continue;
        TileRange tr = tet_tiles(r, B);
        for (int s = lane; s < tr.count; s += 64) {
            int tile;
            if (!tet_tile(r, B, tr, s, tile)) continue;
            // distinct tiles within one tetrahedron: no two lanes share a slot
            const uint32_t slot = lds_bins[tile];
            lds_bins[tile] = slot + 1;
            if (SCATTER) {
                const uint64_t pos = base[(int64_t)tile * B.nseg] + slot;
                if (pos < pair_cap) pairs[pos] = (uint32_t)id;
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
    if (!SCATTER) {
        __syncthreads();
        for (int t = lane; t < ntiles; t += 64) counts[(int64_t)t * B.nseg + seg] = lds_bins[t];
    }
}

hipError_t launch_count(const TetRec *rec, int64_t ntet, const BinParams &B, uint32_t *counts,
                        hipStream_t stream) {
    const size_t lds = sizeof(uint32_t) * (size_t)B.ntx * B.nty;
    hipLaunchKernelGGL((k_bin<false>), dim3(B.nseg), dim3(64), lds, stream, rec, ntet, B, counts,
                       (const uint64_t *)nullptr, (uint32_t *)nullptr, 0ull);
    return hipGetLastError();
}

hipError_t launch_scatter(const TetRec *rec, int64_t ntet, const BinParams &B, const uint64_t *base,
                          uint32_t *pairs, unsigned long long pair_cap, hipStream_t stream) {
    const size_t lds = sizeof(uint32_t) * (size_t)B.ntx * B.nty;
    hipLaunchKernelGGL((k_bin<true>), dim3(B.nseg), dim3(64), lds, stream, rec, ntet, B,
                       (uint32_t *)nullptr, base, pairs, pair_cap);
    return hipGetLastError();
}

// ------------------------------------------------------------------- scan
constexpr int kScanBlock = 1024;
constexpr int kScanPer = 4;
constexpr int kScanTile = kScanBlock * kScanPer;

__device__ inline uint64_t block_exclusive_scan(uint64_t v, uint64_t *sh, uint64_t &total) {
    // sh: kScanBlock / 64 entries
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint64_t incl = v;
    for (int off = 1; off < 64; off <<= 1) {
        const uint64_t o = __shfl_up(incl, off, 64);
        if (lane >= off) incl += o;
    }
    if (lane == 63) sh[wave] = incl;
    __syncthreads();
    if (wave == 0) {
        const int nw = blockDim.x >> 6;
        uint64_t w = lane < nw ? sh[lane] : 0;
        uint64_t wi = w;
        for (int off = 1; off < 64; off <<= 1) {
            const uint64_t o = __shfl_up(wi, off, 64);
            if (lane >= off) wi += o;
        }
        if (lane < nw) sh[lane] = wi - w;
        if (lane == nw - 1) sh[63] = wi;
    }
    __syncthreads();
    total = sh[63];
    const uint64_t r = sh[wave] + incl - v;
    __syncthreads();
    return r;
}

__global__ void __launch_bounds__(kScanBlock) k_scan_reduce(const uint32_t *__restrict__ in,
                                                            int64_t n, uint64_t *__restrict__ sums) {
    __shared__ uint64_t sh[64];
    const int64_t b0 = (int64_t)blockIdx.x * kScanTile;
    uint64_t s = 0;
    for (int q = 0; q < kScanPer; ++q) {
        const int64_t i = b0 + (int64_t)q * kScanBlock + threadIdx.x;
        if (i < n) s += in[i];
    }
    uint64_t total;
    block_exclusive_scan(s, sh, total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

__global__ void __launch_bounds__(kScanBlock) k_scan_sums(uint64_t *__restrict__ sums, int64_t nb) {
    __shared__ uint64_t sh[64];
    uint64_t carry = 0;
    for (int64_t s0 = 0; s0 < nb; s0 += kScanBlock) {
        const int64_t i = s0 + threadIdx.x;
        const uint64_t v = i < nb ? sums[i] : 0;
        uint64_t total;
        const uint64_t ex = block_exclusive_scan(v, sh, total);
        if (i < nb) sums[i] = carry + ex;
        carry += total;
    }
}

__global__ void __launch_bounds__(kScanBlock) k_scan_down(const uint32_t *__restrict__ in, int64_t n,
                                                          const uint64_t *__restrict__ sums,
                                                          uint64_t *__restrict__ out) {
    __shared__ uint64_t sh[64];
    const int64_t b0 = (int64_t)blockIdx.x * kScanTile;
    // each thread owns kScanPer consecutive elements
    const int64_t i0 = b0 + (int64_t)threadIdx.x * kScanPer;
    uint32_t v[kScanPer];
    uint64_t s = 0;
    for (int q = 0; q < kScanPer; ++q) {
        v[q] = (i0 + q < n) ? in[i0 + q] : 0u;
        s += v[q];
    }
    uint64_t total;
    uint64_t run = sums[blockIdx.x] + block_exclusive_scan(s, sh, total);
    for (int q = 0; q < kScanPer; ++q) {
        if (i0 + q < n) out[i0 + q] = run;
        run += v[q];
    }
}

size_t scan_scratch_elems(int64_t n) { return (size_t)((n + kScanTile - 1) / kScanTile) + 1; }

hipError_t launch_scan(const uint32_t *counts, uint64_t *base, int64_t n, uint64_t *scratch,
                       hipStream_t stream) {
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kScanBlock), 0, stream, counts, n, scratch);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kScanBlock), 0, stream, scratch, nb);
    hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nb), dim3(kScanBlock), 0, stream, counts, n, scratch, base);
    return hipGetLastError();
}

// ------------------------------------------------------------------- plan
__device__ inline uint64_t tile_begin(const uint64_t *base, const BinParams &B, int t) {
    return base[(int64_t)t * B.nseg];
}
__device__ inline uint64_t tile_end(const uint64_t *base, const uint32_t *counts, const BinParams &B,
                                    int t, int ntiles) {
    if (t + 1 < ntiles) return base[(int64_t)(t + 1) * B.nseg];
    const int64_t last = (int64_t)ntiles * B.nseg - 1;
    return base[last] + counts[last];
}

__global__ void __launch_bounds__(kScanBlock) k_plan(const uint32_t *__restrict__ counts,
                                                     const uint64_t *__restrict__ base, BinParams B,
                                                     int32_t chunk, uint32_t *__restrict__ tile_items,
                                                     PlanOut *__restrict__ out) {
    __shared__ uint64_t sh[64];
    __shared__ unsigned long long mx;
    const int ntiles = B.ntx * B.nty;
    if (threadIdx.x == 0) mx = 0;
    __syncthreads();
    uint64_t carry = 0;
    for (int t0 = 0; t0 < ntiles; t0 += kScanBlock) {
        const int t = t0 + threadIdx.x;
        uint64_t chunks = 0;
        if (t < ntiles) {
            const uint64_t len = tile_end(base, counts, B, t, ntiles) - tile_begin(base, B, t);
            chunks = (len + chunk - 1) / chunk;
            atomicMax(&mx, (unsigned long long)len);
        }
        uint64_t total;
        const uint64_t ex = block_exclusive_scan(chunks, sh, total);
        if (t < ntiles) tile_items[t] = (uint32_t)(carry + ex);
        carry += total;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        tile_items[ntiles] = (uint32_t)carry;
        out->total_pairs = tile_end(base, counts, B, ntiles - 1, ntiles);
        out->n_items = carry;
        out->max_bin = mx;
    }
}

hipError_t launch_plan(const uint32_t *counts, const uint64_t *base, const BinParams &B,
                       int32_t chunk, uint32_t *tile_items, PlanOut *out, hipStream_t stream) {
    hipLaunchKernelGGL(k_plan, dim3(1), dim3(kScanBlock), 0, stream, counts, base, B, chunk,
                       tile_items, out);
    return hipGetLastError();
}

__global__ void k_items(const uint64_t *__restrict__ base, const uint32_t *__restrict__ tile_items,
                        BinParams B, int32_t chunk, unsigned long long total_pairs,
                        WorkItem *__restrict__ items) {
    const int ntiles = B.ntx * B.nty;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntiles) return;
    const uint64_t b = tile_begin(base, B, t);
    const uint64_t e = t + 1 < ntiles ? tile_begin(base, B, t + 1) : total_pairs;
    const uint32_t first = tile_items[t], n = tile_items[t + 1] - first;
    for (uint32_t c = 0; c < n; ++c) {
        WorkItem w;
        w.first = b + (uint64_t)c * chunk;
        const uint64_t left = e - w.first;
        w.count = (uint32_t)(left < (uint64_t)chunk ? left : (uint64_t)chunk);
        w.tile = (uint32_t)t;
        items[first + c] = w;
    }
}

hipError_t launch_items(const uint64_t *base, const uint32_t *tile_items, const BinParams &B,
                        int32_t chunk, unsigned long long total_pairs, WorkItem *items,
                        hipStream_t stream) {
    const int ntiles = B.ntx * B.nty;
    hipLaunchKernelGGL(k_items, dim3((ntiles + 255) / 256), dim3(256), 0, stream, base, tile_items,
                       B, chunk, total_pairs, items);
    return hipGetLastError();
}

// ----------------------------------------------------------------- raster
// One work item per block.  Tile T x T; every lane owns L consecutive pixels
// of one row (T / L lanes per row), so a block has T*T/L lanes.
// One work item per block.  Records (and FP64 coefficient blocks) are staged
// through LDS in batches of 64 loaded by 64 threads at once, so one memory
// latency covers 64 tetrahedra; every lane then reads each record as an LDS
// broadcast.
constexpr int kBatch = 64;

template <int T, int L, bool COUNT>
__global__ void __launch_bounds__(T * T / L) k_raster(const TetRec *__restrict__ rec,
                                                      const Coef64 *__restrict__ coef64,
                                                      uint32_t coef64_cap,
                                                      const uint32_t *__restrict__ pairs,
                                                      const WorkItem *__restrict__ items, BinParams B,
                                                      double *__restrict__ partials,
                                                      DevCounters *__restrict__ counters) {
    __shared__ TetRec sRec[kBatch];
    __shared__ Coef64 sCoef[kBatch];
    const WorkItem it = items[blockIdx.x];
    const int tid = threadIdx.x;
    const LaneGeom g = lane_geom<T, L>(it.tile, B, tid);
    Acc<L> acc;
    acc.zero();
    unsigned frags = 0, frags4 = 0;
    int since_flush = 0;
    for (uint32_t base = 0; base < it.count; base += kBatch) {
        const uint32_t nb = it.count - base < (uint32_t)kBatch ? it.count - base : (uint32_t)kBatch;
        if (tid < (int)nb) {
            TetRec r;
            r.h.flags = 0;
            const uint32_t id = pairs[it.first + base + tid];
            if (id < B.ntet) {
                r = rec[id];
                if (r.h.flags & REC_FP64) {
                    if (r.h.slot < coef64_cap)
                        sCoef[tid] = coef64[r.h.slot];
                    else
                        r.h.flags = 0;  // slot overflow: the host reruns the call
                }
            }
            sRec[tid] = r;
        }
        __syncthreads();
        for (uint32_t j = 0; j < nb; ++j) {
            const TetRec r = sRec[j];
            if (r.h.flags & REC_VALID) raster_record<L, COUNT>(r, sCoef[j].c, B, g, acc, frags, frags4);
            if (++since_flush == kFlushEvery) {
                acc.flush();
                since_flush = 0;
            }
        }
        __syncthreads();
    }
    acc.flush();
    constexpr int SPR = T / L;
    const int row = tid / SPR, strip = tid % SPR;
    double *out = partials + (size_t)blockIdx.x * (T * T) + (size_t)row * T + strip * L;
#pragma unroll
    for (int k = 0; k < L; ++k) out[k] = acc.d[k];
    if (COUNT) {
        unsigned long long f = wave_sum((unsigned long long)frags);
        unsigned long long f4 = wave_sum((unsigned long long)frags4);
        if ((tid & 63) == 0 && f) atomicAdd(&counters->fragments, f);
        if ((tid & 63) == 0 && f4) atomicAdd(&counters->fragments4, f4);
    }
}

template <int T, int L>
static hipError_t launch_raster_t(const TetRec *rec, const Coef64 *coef64, uint32_t coef64_cap,
                                  const uint32_t *pairs, const WorkItem *items, uint64_t n_items,
                                  const BinParams &B, double *partials, DevCounters *counters,
                                  bool count_fragments, hipStream_t stream) {
    if (n_items == 0) return hipSuccess;
    if (count_fragments)
        hipLaunchKernelGGL((k_raster<T, L, true>), dim3((unsigned)n_items), dim3(T * T / L), 0, stream,
                           rec, coef64, coef64_cap, pairs, items, B, partials, counters);
    else
        hipLaunchKernelGGL((k_raster<T, L, false>), dim3((unsigned)n_items), dim3(T * T / L), 0, stream,
                           rec, coef64, coef64_cap, pairs, items, B, partials, counters);
    return hipGetLastError();
}

hipError_t launch_raster(const TetRec *rec, const Coef64 *coef64, uint32_t coef64_cap,
                         const uint32_t *pairs, const WorkItem *items, uint64_t n_items,
                         const BinParams &B, double *partials, DevCounters *counters,
                         bool count_fragments, hipStream_t stream) {
    switch (B.T) {
        case 16:
            return launch_raster_t<16, 4>(rec, coef64, coef64_cap, pairs, items, n_items, B,
                                          partials, counters, count_fragments, stream);
        case 32:
            return launch_raster_t<32, 16>(rec, coef64, coef64_cap, pairs, items, n_items, B,
                                           partials, counters, count_fragments, stream);
        case 64:
            return launch_raster_t<64, 16>(rec, coef64, coef64_cap, pairs, items, n_items, B,
                                           partials, counters, count_fragments, stream);
        default:
            return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------- finalize
__global__ void k_finalize(const double *__restrict__ partials, const uint32_t *__restrict__ tile_items,
                           BinParams B, float *__restrict__ image) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= (int64_t)B.W * B.H) return;
    const int ix = (int)(p % B.W), iy = (int)(p / B.W);
    const int tile = (iy / B.T) * B.ntx + ix / B.T;
    const int local = (iy % B.T) * B.T + ix % B.T;
    double s = 0.0;
    for (uint32_t it = tile_items[tile]; it < tile_items[tile + 1]; ++it)
        s += partials[(size_t)it * B.T * B.T + local];
    image[p] = (float)s;
}

hipError_t launch_finalize(const double *partials, const uint32_t *tile_items, const BinParams &B,
                           float *image, hipStream_t stream) {
    const int64_t n = (int64_t)B.W * B.H;
    hipLaunchKernelGGL(k_finalize, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, partials,
                       tile_items, B, image);
    return hipGetLastError();
}

// ------------------------------------------------------------ build helpers
__global__ void k_check_finite(const float *__restrict__ x, const float *__restrict__ y,
                               const float *__restrict__ z, int64_t n,
                               unsigned long long *__restrict__ first_bad) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (!isfinite(x[i]) || !isfinite(y[i]) || !isfinite(z[i]))
            atomicMin(first_bad, (unsigned long long)i);
    }
}

hipError_t launch_check_finite(const float *x, const float *y, const float *z, int64_t n,
                               unsigned long long *first_bad, hipStream_t stream) {
    const int64_t want = (n + 255) / 256;
    const int blocks = (int)(want < 16384 ? (want > 0 ? want : 1) : 16384);
    hipLaunchKernelGGL(k_check_finite, dim3(blocks), dim3(256), 0, stream, x, y, z, n, first_bad);
    return hipGetLastError();
}

// Scatter entry s to tracer slot ids[s]; counts how often each slot is hit.
__global__ void k_scatter_ids(const float *__restrict__ x, const float *__restrict__ y,
                              const float *__restrict__ z, const uint64_t *__restrict__ ids,
                              int64_t n, float *__restrict__ ox, float *__restrict__ oy,
                              float *__restrict__ oz, unsigned int *__restrict__ seen,
                              unsigned long long *__restrict__ bad) {
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n;
         s += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t id = ids[s];
        if (id >= (uint64_t)n) {
            atomicMin(bad, (unsigned long long)s);
            continue;
        }
        if (atomicAdd(&seen[id], 1u) != 0u) {
            atomicMin(bad, (unsigned long long)s);
            continue;
        }
        ox[id] = x[s];
        oy[id] = y[s];
        oz[id] = z[s];
    }
}

hipError_t launch_scatter_ids(const float *x, const float *y, const float *z, const uint64_t *ids,
                              int64_t n, float *ox, float *oy, float *oz, unsigned int *seen,
                              unsigned long long *bad, hipStream_t stream) {
    const int64_t want = (n + 255) / 256;
    const int blocks = (int)(want < 16384 ? (want > 0 ? want : 1) : 16384);
    hipLaunchKernelGGL(k_scatter_ids, dim3(blocks), dim3(256), 0, stream, x, y, z, ids, n, ox, oy,
                       oz, seen, bad);
    return hipGetLastError();
}

}  // namespace tess
