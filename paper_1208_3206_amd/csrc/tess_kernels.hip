// HIP kernels of the tessellation projector (gfx950).
//
// Pipeline of one projection (all on the caller's stream):
//   k_setup    one thread per lattice cube: gather the 8 corners (coalesced
//              SoA loads), unwrap them to the periodic image nearest corner 0,
//              cut the cube into the six tetrahedra of the connectivity table,
//              compute the volume determinant (Eq. Eqn:TetVolume; FP32, redone
//              in FP64 when flagged) and the tetrahedron's screen footprint in
//              FP64 (record head + coefficients)
//   k_bin      per segment of tetrahedra: count, then scatter, the ids into
//              per-tile lists (tiles are bands of Th rows x Tw columns)
//   k_scan     exclusive scan of the (tile, segment) counts
//   k_plan     per-tile lists split into raster work items of <= chunk entries
//   k_raster   per work item: the tile's second-difference array lives in LDS;
//              every lane takes whole tetrahedra and adds, for each pixel row
//              they cross, the few break-point terms of the row's piecewise
//              linear footprint (LDS FP64 atomics); the tile is then added to
//              the image-sized FP64 array in HBM
//   k_finalize per image row: two running sums of that array -> FP32 image
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
// centres exactly on it.  Along a pixel row the pyramid is piecewise linear,
// so the raster works on second differences of rows instead of on pixels:
// its cost is per (tetrahedron, row), not per covered pixel.
#include "tess_tet.h"

#include <algorithm>
#include <cfloat>
#include <climits>
#include <mutex>

namespace tess {


__device__ inline unsigned long long wave_sum(unsigned long long v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// One thread per lattice cube; writes the six records 6*cube .. 6*cube+5
// (edge form: the edge slots of the tetrahedra that edge_tet_fast settles,
// the others left to k_setup_rest).  Two wavefronts per SIMD at least: the
// general setup would otherwise take 256 VGPRs and run one wavefront per
// SIMD.  The edge form's kernel indexes no array by tetrahedron and takes
// no scratch memory, which would cap the wavefronts in flight.
template <int FORM, bool EDGES>
__global__ void __launch_bounds__(256, 2) k_setup(LatticeParams L, ViewParams V,
                                               RecHead *__restrict__ head,
                                               Payload *__restrict__ coef,
                                               DevCounters *__restrict__ counters) {
    CubeCounts cnt;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int lane = threadIdx.x & 63;
    if constexpr (EDGES) {
        // edge form, the common cases of every tetrahedron (its creases to
        // the edge slots, or a line-form record of its own, stored compactly
        // as it comes); the others, and line-form records that found no
        // room, are marked in the spill bit set, which k_setup_rest reads
        // next
        for (int64_t cube = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; cube < L.ncubes; cube += stride) {
            uint32_t todo = 0u;
            setup_cube<FORM, EDGES, 1>(
                L, V, cube, [](int, const RecHead &, const Payload &) {}, cnt, &todo,
                [&](int t, const RecHead &R) -> Payload * {
                    // a line-form record: its slot first, then its values
                    // straight to memory (held in registers they would cost
                    // the kernel its occupancy)
                    const unsigned long long slot = atomicAdd(V.own, 1ull);
                    if (slot < V.own_cap) {
                        head[slot] = R;
                        return &coef[slot];
                    }
                    // no room: the count taken back (it stays at or above the
                    // capacity, so no slot below it is handed out twice); the
                    // tetrahedron is marked for k_setup_rest, which counts it
                    // and marks it again
                    atomicAdd(V.own, ~0ull);
                    return nullptr;
                },
                [](int) {});
            while (todo) {
                const int t = __builtin_ctz(todo);
                todo &= todo - 1u;
                const int64_t tet = 6 * cube + t;
                atomicOr(&V.spill[tet >> 5], 1u << (tet & 31));
            }
        }
    } else {
        // The block's heads are built in LDS and then written as one
        // contiguous run: a thread's six 16-byte heads written in place would
        // make every store instruction touch 64 lines a quarter each (partial
        // lines cost a read-modify-write in HBM).  Payloads are written in
        // place as they are built (holding six 144-byte records in registers
        // would cost the occupancy; they are whole 128-byte lines).
        __shared__ RecHead sh_head[6 * 256];
        for (int64_t first = (int64_t)blockIdx.x * blockDim.x; first < L.ncubes; first += stride) {
            const int64_t cube = first + threadIdx.x;
            if (cube < L.ncubes)
                setup_cube<FORM, EDGES>(
                    L, V, cube,
                    [&](int t, const RecHead &R, const Payload &P) {
                        sh_head[6 * threadIdx.x + t] = R;
                        if (R.flags & REC_VALID) coef[6 * cube + t] = P;  // nothing reads other payloads
                    },
                    cnt);
            __syncthreads();
            const int nh = 6 * (int)(L.ncubes - first < 256 ? L.ncubes - first : 256);
            for (int i = threadIdx.x; i < nh; i += 256) head[6 * first + i] = sh_head[i];
            __syncthreads();
        }
    }
    const unsigned long long n_tets = wave_sum(cnt.n_tets), n_zero = wave_sum(cnt.n_zero),
                             n_inv = wave_sum(cnt.n_inv), n_dets = wave_sum(cnt.n_dets),
                             n_deg = wave_sum(cnt.n_deg);
    if (lane == 0) {
        if (n_tets) atomicAdd(&counters->tets, n_tets);
        if (n_zero) atomicAdd(&counters->zero_volume, n_zero);
        if (n_inv) atomicAdd(&counters->inverted, n_inv);
        if (n_dets) atomicAdd(&counters->fp64_dets, n_dets);
        if (n_deg) atomicAdd(&counters->degenerate, n_deg);
    }
}

// Edge form, after k_setup: the tetrahedra it left to the general code, one
// thread per 32-bit word of the spill bit set (the bits k_setup marked).  A
// word is cleared, then each of its tetrahedra set up; those whose own
// record finds no room mark their bit again, the set's meaning for the
// raster (every tetrahedron in one word belongs to this thread).
__global__ void __launch_bounds__(256) k_setup_rest(LatticeParams L, ViewParams V, RecHead *__restrict__ head,
                                                    Payload *__restrict__ coef, DevCounters *__restrict__ counters) {
    CubeCounts cnt;
    const int64_t nwords = (6 * L.ncubes + 31) / 32;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w < nwords; w += stride) {
        uint32_t bits = V.spill[w];
        if (bits == 0u) continue;
        V.spill[w] = 0u;
        while (bits) {
            const int b = __builtin_ctz(bits);
            bits &= bits - 1u;
            const int64_t tet = 32 * w + b;
            const int64_t cube = tet / 6;
            uint32_t todo = 1u << (int)(tet - 6 * cube);
            setup_cube<kFormPyramid, true, 2>(
                L, V, cube,
                [&](int t, const RecHead &R, const Payload &P) {
                    if (!(R.flags & REC_VALID)) return;
                    const unsigned long long slot = atomicAdd(V.own, 1ull);
                    if (slot < V.own_cap) {
                        head[slot] = R;
                        coef[slot] = P;
                    } else {
                        const int64_t id = 6 * cube + t;
                        atomicOr(&V.spill[id >> 5], 1u << (id & 31));
                    }
                },
                cnt, &todo);
        }
    }
    const unsigned long long n_tets = wave_sum(cnt.n_tets), n_zero = wave_sum(cnt.n_zero),
                             n_inv = wave_sum(cnt.n_inv), n_dets = wave_sum(cnt.n_dets),
                             n_deg = wave_sum(cnt.n_deg);
    if ((threadIdx.x & 63) == 0) {
        if (n_tets) atomicAdd(&counters->tets, n_tets);
        if (n_zero) atomicAdd(&counters->zero_volume, n_zero);
        if (n_inv) atomicAdd(&counters->inverted, n_inv);
        if (n_dets) atomicAdd(&counters->fp64_dets, n_dets);
        if (n_deg) atomicAdd(&counters->degenerate, n_deg);
    }
}

// Edge form: one thread per lattice vertex, its seven edge records after
// the tetrahedra's (ids own_cap + tau nvert + v).
__global__ void __launch_bounds__(256) k_edges(LatticeParams L, ViewParams V, RecHead *__restrict__ head,
                                               EdgePayload *__restrict__ ecoef) {
    const int64_t nv = (int64_t)L.d[0] * L.d[1] * L.d[2];
    const int64_t first = (int64_t)V.own_cap;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nv; v += stride)
        setup_vertex_edges(L, V, v, head + first + v, ecoef + v);
}

hipError_t launch_edges(const LatticeParams &L, const ViewParams &V, RecHead *head, EdgePayload *ecoef,
                        hipStream_t stream) {
    const int64_t nv = (int64_t)L.d[0] * L.d[1] * L.d[2];
    const int64_t want = (nv + 255) / 256;
    const int blocks = (int)(want < 65536 ? (want > 0 ? want : 1) : 65536);
    hipLaunchKernelGGL(k_edges, dim3(blocks), dim3(256), 0, stream, L, V, head, ecoef);
    return hipGetLastError();
}

// One thread per cube: the integral of the projected value q over all
// tetrahedra, the image's scale for the crease threshold when q != rho.
__global__ void __launch_bounds__(256) k_qsum(LatticeParams L, ViewParams V, double *__restrict__ qsum) {
    double sum = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t cube = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; cube < L.ncubes; cube += stride)
        sum += cube_qvol(L, V, cube);
    for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off, 64);
    if ((threadIdx.x & 63) == 0 && sum != 0.0) atomicAdd(qsum, sum);
}

// Blocks of 256 threads for a grid-stride loop over n items: at most
// kCubeBlocks, so that a thread takes several cubes.  One cube per thread
// ran a quarter of a million short wavefronts per frame at 256^3, whose
// start-up and end-of-wavefront counter atomics (all on the same few
// addresses) took longer than the setup's arithmetic.
constexpr int kCubeBlocks = 8192;
inline int cube_blocks(int64_t n, int cap = kCubeBlocks) {
    const int64_t want = (n + 255) / 256;
    return (int)(want < cap ? (want > 0 ? want : 1) : cap);
}

hipError_t launch_qsum(const LatticeParams &L, const ViewParams &V, double *qsum, hipStream_t stream) {
    const int blocks = cube_blocks(L.ncubes);
    hipLaunchKernelGGL(k_qsum, dim3(blocks), dim3(256), 0, stream, L, V, qsum);
    return hipGetLastError();
}

hipError_t launch_setup(const LatticeParams &L, const ViewParams &V, RecHead *head, Payload *coef,
                        DevCounters *counters, hipStream_t stream) {
    const int blocks = cube_blocks(L.ncubes);
    switch (view_form(V)) {
        case kFormFace:
            hipLaunchKernelGGL((k_setup<kFormFace, false>), dim3(blocks), dim3(256), 0, stream, L, V, head, coef, counters);
            break;
        case kFormSplat:
            hipLaunchKernelGGL((k_setup<kFormSplat, false>), dim3(blocks), dim3(256), 0, stream, L, V, head, coef,
                               counters);
            break;
        case kFormPersp:
            hipLaunchKernelGGL((k_setup<kFormPersp, false>), dim3(blocks), dim3(256), 0, stream, L, V, head, coef,
                               counters);
            break;
        default:
            if (V.edges) {
                hipLaunchKernelGGL((k_setup<kFormPyramid, true>), dim3(blocks), dim3(256), 0, stream, L, V, head,
                                   coef, counters);
                hipLaunchKernelGGL(k_setup_rest, dim3(cube_blocks((6 * L.ncubes + 31) / 32, 1024)), dim3(256), 0,
                                   stream, L, V, head, coef, counters);
            } else
                hipLaunchKernelGGL((k_setup<kFormPyramid, false>), dim3(blocks), dim3(256), 0, stream, L, V, head,
                                   coef, counters);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------- binning
// One block per segment of seg_len consecutive tetrahedra; lanes take
// tetrahedra in turn and count (or place) them in an LDS array of per-tile
// counters.  The order inside one segment's share of a tile list follows the
// atomics; the raster's sums do not depend on it beyond rounding.  With
// nkey > 1 each placed id carries the pair's work class in its top bits.
//
// The scatter stages a segment's ids in LDS, sorted by tile (a counting sort
// on this segment's counts from the count pass), then copies each tile's run
// to its place in the pair list: whole runs instead of single 4-byte writes
// all over the list.  A segment with more pairs than the stage holds writes
// its ids directly.
constexpr int kBinBlock = 512;
constexpr int kStage = 16384;     // staged pair ids per segment (64 KiB of LDS)

// Exclusive scan of v over the block's kBinBlock threads (sh: kBinBlock / 64 + 1 words).
__device__ inline uint32_t bin_block_scan(uint32_t v, uint32_t *sh, uint32_t &total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t incl = v;
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t o = __shfl_up(incl, off, 64);
        if (lane >= off) incl += o;
    }
    if (lane == 63) sh[wave] = incl;
    __syncthreads();
    uint32_t before = 0, all = 0;
    for (int w = 0; w < kBinBlock / 64; ++w) {
        before += w < wave ? sh[w] : 0u;
        all += sh[w];
    }
    __syncthreads();
    total = all;
    return before + incl - v;
}

template <bool SCATTER>
__global__ void __launch_bounds__(kBinBlock) k_bin(const RecHead *__restrict__ head, int64_t ntet,
                                                   BinParams B, uint32_t *__restrict__ counts,
                                                   const uint64_t *__restrict__ base,
                                                   uint32_t *__restrict__ pairs,
                                                   unsigned long long pair_cap, int staged) {
    extern __shared__ uint32_t lds_bins[];  // per tile: count, or next slot; then (staged) the stage
    __shared__ uint32_t sh_scan[kBinBlock / 64 + 1];
    const int ntiles = B.ntx * B.nty;
    const int seg = blockIdx.x;
    uint32_t *stage = lds_bins + ntiles;
    // scatter: each tile's counter starts at this segment's first slot: in the
    // stage (its offset among this segment's pairs), or as an absolute
    // position when every pair fits 32 bits (no base read per pair), else
    // relative to the tile's start
    bool use_stage = false;
    if (SCATTER && staged) {
        // this segment's pairs per tile (from the count pass), scanned
        const int per = (ntiles + kBinBlock - 1) / kBinBlock;
        const int t0 = threadIdx.x * per;
        uint32_t mine = 0;
        for (int k = 0; k < per; ++k)
            if (t0 + k < ntiles) mine += counts[(int64_t)(t0 + k) * B.nseg + seg];
        uint32_t total;
        uint32_t run = bin_block_scan(mine, sh_scan, total);
        use_stage = total <= (uint32_t)kStage;  // the same for the whole block
        if (use_stage)
            for (int k = 0; k < per; ++k)
                if (t0 + k < ntiles) {
                    const uint32_t c = counts[(int64_t)(t0 + k) * B.nseg + seg];
                    lds_bins[t0 + k] = run;
                    run += c;
                }
    }
    const bool abs32 = SCATTER && pair_cap <= 0xffffffffull;
    if (!use_stage)
        for (int t = threadIdx.x; t < ntiles; t += kBinBlock) {
            if (SCATTER)
                lds_bins[t] = abs32 ? (uint32_t)base[(int64_t)t * B.nseg + seg]
                                    : (uint32_t)(base[(int64_t)t * B.nseg + seg] - base[(int64_t)t * B.nseg]);
            else
                lds_bins[t] = 0;
        }
    __syncthreads();
    const int64_t t0 = (int64_t)seg * B.seg_len;
    const int64_t t1 = min(ntet, t0 + B.seg_len);
    for (int64_t id = t0 + threadIdx.x; id < t1; id += kBinBlock) {
        const RecHead r = head[id];
        if (!(r.flags & REC_VALID)) continue;
        const TileRange tr = tet_tiles(r, B);
        ClassRows cr;
        cr.crease = false;
        if (SCATTER && B.nkey > 1) cr = class_rows(r);
        for (int sy = 0; sy < tr.cy; ++sy) {
            const int ty = tr.sy + sy < B.nty ? tr.sy + sy : tr.sy + sy - B.nty;
            const uint32_t tag = SCATTER && B.nkey > 1 ? (uint32_t)row_class(cr, r, B, ty) << kClassShift : 0u;
            for (int sx = 0; sx < tr.cx; ++sx) {
                const int tile = ty * B.ntx + (tr.sx + sx < B.ntx ? tr.sx + sx : tr.sx + sx - B.ntx);
                const uint32_t slot = atomicAdd(&lds_bins[tile], 1u);
                if (SCATTER) {
                    if (use_stage) {
                        if (slot < (uint32_t)kStage) stage[slot] = (uint32_t)id | tag;
                    } else {
                        const uint64_t pos = abs32 ? (uint64_t)slot : base[(int64_t)tile * B.nseg] + slot;
                        if (pos < pair_cap) pairs[pos] = (uint32_t)id | tag;
                    }
                }
            }
        }
    }
    if (SCATTER && use_stage) {
        // each wavefront copies whole tile runs: the run of tile t ends at
        // lds_bins[t] (its cursor) and has counts[t][seg] entries
        __syncthreads();
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        for (int t = wave; t < ntiles; t += kBinBlock / 64) {
            const uint32_t c = counts[(int64_t)t * B.nseg + seg];
            if (c == 0) continue;
            const uint32_t first = lds_bins[t] - c;
            const uint64_t dst = base[(int64_t)t * B.nseg + seg];
            for (uint32_t j = lane; j < c; j += 64)
                if (dst + j < pair_cap) pairs[dst + j] = stage[first + j];
        }
    }
    if (!SCATTER) {
        __syncthreads();
        for (int t = threadIdx.x; t < ntiles; t += kBinBlock) counts[(int64_t)t * B.nseg + seg] = lds_bins[t];
    }
}

// one 32-bit LDS counter per tile, in both passes; the scatter's stage
// beside them while the counters leave room for it in 96 KiB
static bool bin_staged(const BinParams &B) { return (size_t)B.ntx * B.nty + kStage <= 24576; }
static size_t bin_lds_bytes(const BinParams &B, bool scatter) {
    return sizeof(uint32_t) * ((size_t)B.ntx * B.nty + (scatter && bin_staged(B) ? kStage : 0));
}

hipError_t launch_count(const RecHead *head, int64_t ntet, const BinParams &B, uint32_t *counts,
                        hipStream_t stream) {
    const size_t lds = bin_lds_bytes(B, false);
    hipLaunchKernelGGL((k_bin<false>), dim3(B.nseg), dim3(kBinBlock), lds, stream, head, ntet, B, counts,
                       (const uint64_t *)nullptr, (uint32_t *)nullptr, 0ull, 0);
    return hipGetLastError();
}

hipError_t launch_scatter(const RecHead *head, int64_t ntet, const BinParams &B, const uint32_t *counts,
                          const uint64_t *base, uint32_t *pairs, unsigned long long pair_cap, hipStream_t stream) {
    const size_t lds = bin_lds_bytes(B, true);
    hipLaunchKernelGGL((k_bin<true>), dim3(B.nseg), dim3(kBinBlock), lds, stream, head, ntet, B,
                       const_cast<uint32_t *>(counts), base, pairs, pair_cap, bin_staged(B) ? 1 : 0);
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

__global__ void __launch_bounds__(kScanBlock) k_totals(const uint32_t *__restrict__ counts,
                                                       const uint64_t *__restrict__ base, BinParams B,
                                                       unsigned long long cap, PlanOut *__restrict__ out,
                                                       unsigned int *__restrict__ overflow) {
    __shared__ unsigned long long mx;
    const int ntiles = B.ntx * B.nty;
    if (threadIdx.x == 0) mx = 0;
    __syncthreads();
    for (int t = threadIdx.x; t < ntiles; t += kScanBlock) {
        const uint64_t len = tile_end(base, counts, B, t, ntiles) - tile_begin(base, B, t);
        atomicMax(&mx, (unsigned long long)len);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned long long total = tile_end(base, counts, B, ntiles - 1, ntiles);
        out->total_pairs = total;
        out->max_bin = mx;
        out->n_items = 0;
        if (total > cap && overflow) atomicOr(overflow, 1u);
    }
}

hipError_t launch_totals(const uint32_t *counts, const uint64_t *base, const BinParams &B,
                         unsigned long long cap, PlanOut *out, unsigned int *overflow, hipStream_t stream) {
    hipLaunchKernelGGL(k_totals, dim3(1), dim3(kScanBlock), 0, stream, counts, base, B, cap, out, overflow);
    return hipGetLastError();
}

// A list longer than the pair buffer (cap) gets no work items: the image is
// then left unrastered and its PlanOut shows total_pairs > cap.
__global__ void __launch_bounds__(kScanBlock) k_plan(const uint32_t *__restrict__ counts,
                                                     const uint64_t *__restrict__ base, BinParams B,
                                                     int32_t chunk, unsigned long long cap,
                                                     uint32_t *__restrict__ tile_items,
                                                     PlanOut *__restrict__ out) {
    __shared__ uint64_t sh[64];
    const int ntiles = B.ntx * B.nty;
    const bool fits = tile_end(base, counts, B, ntiles - 1, ntiles) <= cap;
    uint64_t carry = 0;
    for (int t0 = 0; t0 < ntiles; t0 += kScanBlock) {
        const int t = t0 + threadIdx.x;
        uint64_t chunks = 0;
        if (t < ntiles && fits) {
            const uint64_t len = tile_end(base, counts, B, t, ntiles) - tile_begin(base, B, t);
            chunks = (len + chunk - 1) / chunk;
        }
        uint64_t total;
        const uint64_t ex = block_exclusive_scan(chunks, sh, total);
        if (t < ntiles) tile_items[t] = (uint32_t)(carry + ex);
        carry += total;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        tile_items[ntiles] = (uint32_t)carry;
        out->n_items = carry;
    }
}

hipError_t launch_plan(const uint32_t *counts, const uint64_t *base, const BinParams &B,
                       int32_t chunk, unsigned long long cap, uint32_t *tile_items, PlanOut *out,
                       hipStream_t stream) {
    hipLaunchKernelGGL(k_plan, dim3(1), dim3(kScanBlock), 0, stream, counts, base, B, chunk, cap,
                       tile_items, out);
    return hipGetLastError();
}

__global__ void k_items(const uint64_t *__restrict__ base, const uint32_t *__restrict__ tile_items,
                        BinParams B, int32_t chunk, const PlanOut *__restrict__ plan,
                        WorkItem *__restrict__ items) {
    const int ntiles = B.ntx * B.nty;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntiles) return;
    const uint64_t b = tile_begin(base, B, t);
    const uint64_t e = t + 1 < ntiles ? tile_begin(base, B, t + 1) : plan->total_pairs;
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
                        int32_t chunk, const PlanOut *plan, WorkItem *items, hipStream_t stream) {
    const int ntiles = B.ntx * B.nty;
    hipLaunchKernelGGL(k_items, dim3((ntiles + 255) / 256), dim3(256), 0, stream, base, tile_items,
                       B, chunk, plan, items);
    return hipGetLastError();
}

__global__ void k_zero(double *__restrict__ p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

hipError_t launch_zero(double *p, int64_t n, hipStream_t stream) {
    const int64_t want = (n + 255) / 256;
    const int blocks = (int)(want < 8192 ? (want > 0 ? want : 1) : 8192);
    hipLaunchKernelGGL(k_zero, dim3(blocks), dim3(256), 0, stream, p, n);
    return hipGetLastError();
}

// ----------------------------------------------------------------- raster
// One work item per block.  The block holds the tile's second-difference
// array A[Th][Tw] (FP64) in LDS; lanes take the item's tetrahedra in turn
// and add each pixel row's break-point terms with LDS atomics.  At the end
// the tile is added to the image-sized array `acc` (FP64 atomics in L2; a
// tile has several items).
constexpr int kPad = 2;
constexpr int kIdBurst = 8;     // pair ids a lane loads at once
constexpr int kSortPer = 7;     // pair ids per lane in one wavefront's class sort
constexpr int kNumClasses = 32;
constexpr size_t kLdsBytes = 160 * 1024 - 64;  // dynamic LDS: 64 bytes stay for the static counter
// edge form: a wavefront's queue of pairs whose seam lines are still to draw
// (at most 63 waiting plus 64 added in one round)
constexpr int kSeamQueue = 128;
// Row stride of the tile accumulator: Tw + 4 cells; for the edge form
// (`banked`) rounded up to 3 modulo 32 doubles.  A 16-lane group adds to
// 16 consecutive rows at columns x0 + floor(r s), s the edge's columns per
// row, so lane r's cell lies r (3 + s) doubles (mod 32) from lane 0's: 16
// different banks for s = 0 and s = -1, the slopes of two of the lattice's
// seven edge kinds seen along an axis, and two lanes a bank for s = +1.  (At
// 1 modulo 32, s = -1 put all 16 in one bank; measured at stress 2048^2 the
// raster took 24.2 ms there, 22.2 ms at 3, 22.3-22.6 at 5, 7, 9 and 11.)
// The rounded rows leave room for one copy of the seam lines and the seam
// queues of a 1024-thread block.  (The other forms draw a record per lane,
// at cells with no such pattern, and need the LDS for the wavefronts' class
// sorts.)
__host__ __device__ inline int tile_stride(int Tw, int Th, bool banked) {
    const int plain = Tw + 2 * kPad, padded = ((plain + 28) & ~31) + 3;
    const size_t need = sizeof(double) * ((size_t)Th * padded + 2 * (size_t)Th + 3 * ((size_t)Th + 1)) +
                        sizeof(uint32_t) * 16 * kSeamQueue;
    return banked && need <= kLdsBytes ? padded : plain;
}

__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// min(max(x, lo), hi) for lo <= hi in one instruction (the compiler forms
// v_med3_i32 only for constant bounds).
__device__ __forceinline__ int med3_i32(int x, int lo, int hi) {
    int r;
    asm volatile("v_med3_i32 %0, %1, %2, %3" : "=v"(r) : "v"(x), "v"(lo), "v"(hi));
    return r;
}

// Lane I's value of its 16-lane row, in every lane of the row (a DPP row
// broadcast: no LDS traffic).
template <int I>
__device__ __forceinline__ uint32_t row_bcast(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x150 + I, 0xf, 0xf, true);
}
template <int I>
__device__ __forceinline__ double row_bcast(double x) {
    const uint64_t b = (uint64_t)__double_as_longlong(x);
    const uint64_t lo = row_bcast<I>((uint32_t)b), hi = row_bcast<I>((uint32_t)(b >> 32));
    return __longlong_as_double((long long)(lo | (hi << 32)));
}

// A double in LDS addressed by its byte offset: the kink loop clamps cell
// addresses, not column indices, and the atomics take them as they are.
typedef __attribute__((address_space(3))) double lds_f64;

// The kinks of the edge jobs of a 16-lane group, edge I first: its rows
// r0 + s, s = q, q + 16, ... < cnt, on lane q (pk: cnt << 8), into the tile
// rows of stride8 bytes.  Each kink's terms are edge_pair's: crossing u =
// fma(r, sl, base), D (1 - f) at tile column clamp(floor(u) - shift) + 1 and
// D f beside it.  The job's owner lane precomputed the LDS byte offsets of
// its first tile row: p1 of record column 0 (so that floor(u) * 8 + p1 is
// the first cell) and p2 of the row's first padding cell (the clamp's lower
// end; its upper end n8 bytes on); qs8 moves them to lane q's row.  TWO:
// every job has at most 32 rows (tiles of at most 32 rows), two steps
// unrolled.
template <int I, bool TWO>
__device__ __forceinline__ void group_kinks(const EdgeJob &J, uint32_t pk, uint32_t p1, uint32_t p2, int q, int qs8,
                                            int n8, int stride8) {
    const uint32_t pki = row_bcast<I>(pk);
    const int cnt = (int)(pki >> 8);
    if (__builtin_amdgcn_ballot_w64(cnt > q) != 0ull) {  // some group has rows of its edge I
        const int r0 = (int)row_bcast<I>((uint32_t)J.r0);
        const int rowp = (int)row_bcast<I>(p1) + qs8, lo = (int)row_bcast<I>(p2) + qs8;
        const double base = row_bcast<I>(J.base), sl = row_bcast<I>(J.sl), D = row_bcast<I>(J.D);
        auto kink = [&](int rowb, int lob, double rv) {
            const double u = fma(rv, sl, base);
            const double fl = floor(u);
            lds_f64 *const c = (lds_f64 *)(uintptr_t)(uint32_t)med3_i32(((int)fl << 3) + rowb, lob, lob + n8);
            const double v1 = fma(D, fl - u, D);
            __hip_atomic_fetch_add(c, v1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            __hip_atomic_fetch_add(c + 1, D - v1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        };
        if constexpr (TWO) {
            const double rv = (double)(r0 + q);
            if (q < cnt) kink(rowp, lo, rv);
            if (q + 16 < cnt) kink(rowp + 16 * stride8, lo + 16 * stride8, rv + 16.0);
        } else {
            int rb = rowp, lb = lo;
            for (int s = q; s < cnt; s += 16, rb += 16 * stride8, lb += 16 * stride8) kink(rb, lb, (double)(r0 + s));
        }
    }
    if constexpr (I < 15) group_kinks<I + 1, TWO>(J, pk, p1, p2, q, qs8, n8, stride8);
}

// LDS of one wavefront's class sort: kNumClasses counters, then 64 * kSortPer entries
constexpr int kSortWords = kNumClasses + 64 * kSortPer;

template <int TPB, int FORM, bool COUNT = true>
__global__ void __launch_bounds__(TPB) k_raster(const RecHead *__restrict__ head,
                                                const Payload *__restrict__ coef,
                                                const EdgePayload *__restrict__ ecoef,
                                                const uint32_t *__restrict__ pairs,
                                                const WorkItem *__restrict__ items,
                                                const PlanOut *__restrict__ plan, BinParams B, int sorted,
                                                double *__restrict__ acc,
                                                DevCounters *__restrict__ counters) {
    extern __shared__ double sA[];
    if ((unsigned long long)blockIdx.x >= plan->n_items) return;
    const WorkItem it = items[blockIdx.x];
    const int tx = (int)(it.tile % (uint32_t)B.ntx), ty = (int)(it.tile / (uint32_t)B.ntx);
    const int tx0 = tx * B.Tw, ty0 = ty * B.Th;
    const int n = min(B.Tw, B.W - tx0), rows = min(B.Th, B.H - ty0);
    // rows of at least Tw + 4 cells: two padding cells each side take the adds that
    // fall outside the tile, so that the raster needs no bounds tests
    const int stride = tile_stride(B.Tw, B.Th, FORM == kFormEdge);
    const int tsize = B.Th * stride;
    auto cell = [&](int row, int j) { return row * stride + kPad + j; };
    // then (edge form under wrap) per tile row the seam line a + b j, in
    // seam_copies copies (lane t adds to copy t % seam_copies: the lanes of a
    // 16-lane group draw 16 neighbouring edges over the same rows, and adds
    // of one instruction to one cell are serialised); a values, then b
    // then the range updates of the seam lines in difference form, Th + 1
    // cells each (added at a range's first row, taken off after its last):
    // alpha, beta (a += alpha + beta rho) and gamma (b += gamma), in
    // seam_copies copies too
    double *sSeam = sA + tsize;
    const int nsc = B.seam ? B.seam_copies : 0;
    const int nseam = (2 * B.Th + 3 * (B.Th + 1)) * nsc;
    const int sc = nsc ? (int)(threadIdx.x % (unsigned)nsc) : 0;
    double *sDiff = sSeam + 2 * B.Th * nsc;
    const int dstride = (B.Th + 1) * nsc;  // one difference array (all copies)
    for (int i = threadIdx.x; i < tsize + nseam; i += TPB) sA[i] = 0.0;
    __shared__ uint32_t s_next;  // edge form: chunks handed out so far
    if (threadIdx.x == 0) s_next = 0u;
    __syncthreads();
    long long frags = 0;  // edge records add signed terms
    uint32_t spans = 0, kinks = 0;
    auto seam_range = [&](int lo, int hi, double alpha, double beta, double gamma) {
        atomicAdd(&sDiff[lo * nsc + sc], alpha);
        atomicAdd(&sDiff[(hi + 1) * nsc + sc], -alpha);
        atomicAdd(&sDiff[dstride + lo * nsc + sc], beta);
        atomicAdd(&sDiff[dstride + (hi + 1) * nsc + sc], -beta);
        atomicAdd(&sDiff[2 * dstride + lo * nsc + sc], gamma);
        atomicAdd(&sDiff[2 * dstride + (hi + 1) * nsc + sc], -gamma);
    };
    auto one = [&](uint32_t id) {
        if (id >= B.ntet) return;
        if constexpr (FORM == kFormEdge) {
            // an edge record: its half line is all the raster reads
            if (id >= B.first_edge) {
                frags += (int32_t)edge_pair<COUNT>(
                    ecoef[id - B.first_edge], id - B.first_edge, COUNT ? head[id].spare : 0u, B, tx0, ty0, n, rows,
                    [&](int row, int j, double v1, double v2) {
                        const int x = cell(row, j);
                        atomicAdd(&sA[x], v1);
                        atomicAdd(&sA[x + 1], v2);
                    },
                    [&](int row, double a, double b) {
                        atomicAdd(&sSeam[row * nsc + sc], a);
                        atomicAdd(&sSeam[(B.Th + row) * nsc + sc], b);
                    },
                    seam_range, kinks);
                return;
            }
        }
        const RecHead h = coef[id].h;
        if (!(h.flags & REC_VALID)) return;
        frags += (int32_t)raster_record<FORM>(
            h, coef[id].c, B, tx0, ty0, n, rows,
            [&](int row, int j, double v) { atomicAdd(&sA[cell(row, j)], v); },
            [&](int row, double a, double b) {
                atomicAdd(&sSeam[row * nsc + sc], a);
                atomicAdd(&sSeam[(B.Th + row) * nsc + sc], b);
            },
            spans, kinks);
    };
    // lane t takes entries t*per .. t*per+per-1: the list is in rough id order
    // (neighbouring cubes), so this spreads a wavefront's 64 footprints over
    // the tile instead of stacking their atomics on the same LDS cells
    const uint32_t per = (it.count + TPB - 1) / TPB;
    const uint32_t e0 = threadIdx.x * per, e1 = min(it.count, e0 + per);
    if constexpr (FORM == kFormPersp) {
        // per pixel, and a footprint may fill the tile: each wavefront takes
        // its share of the list one pair at a time, its 64 lanes striding over
        // the pair's pixels
        const uint32_t nw = TPB / 64, lane = threadIdx.x & 63u;
        const uint32_t wper = (it.count + nw - 1) / nw;
        const uint32_t w0 = (threadIdx.x >> 6) * wper, w1 = min(it.count, w0 + wper);
        for (uint32_t e = w0; e < w1; ++e) {
            const uint32_t id = pairs[it.first + e];
            if (id >= B.ntet) continue;
            const RecHead h = coef[id].h;
            if (!(h.flags & REC_VALID)) continue;
            frags += persp_pair(h, coef[id].c, B, tx0, ty0, n, rows, (int)lane, 64,
                                [&](int row, int j, double v) { atomicAdd(&sA[cell(row, j)], v); },
                                spans, kinks);
        }
    } else if (FORM == kFormPyramid && sorted) {
        // The wavefront takes the next kSortPer entries of each of its lanes'
        // slices and deals them back out in work-class order (a counting sort
        // in its own LDS area): the lanes that step through their creases
        // together then hold pairs of about the same work.  `per` is the same
        // for every lane, so the whole wavefront runs every round.
        const uint32_t lane = threadIdx.x & 63u;
        uint32_t *cnt = reinterpret_cast<uint32_t *>(sA + tsize + nseam) + (threadIdx.x >> 6) * kSortWords;
        uint32_t *ent = cnt + kNumClasses;
        for (uint32_t b = 0; b < per; b += kSortPer) {
            uint32_t v[kSortPer], rk[kSortPer];
#pragma unroll
            for (int i = 0; i < kSortPer; ++i) {
                const uint32_t e = e0 + b + (uint32_t)i;
                v[i] = (b + (uint32_t)i < per && e < e1) ? pairs[it.first + e] : kIdMask;  // empty: class 0
            }
            if (lane < (uint32_t)kNumClasses) cnt[lane] = 0u;
            wave_sync();
#pragma unroll
            for (int i = 0; i < kSortPer; ++i) rk[i] = atomicAdd(&cnt[v[i] >> kClassShift], 1u);
            wave_sync();
            // class offsets: exclusive prefix sum of the counts over the lanes
            const uint32_t c = lane < (uint32_t)kNumClasses ? cnt[lane] : 0u;
            uint32_t incl = c;
#pragma unroll
            for (int off = 1; off < kNumClasses; off <<= 1) {
                const uint32_t o = __shfl_up(incl, off, 64);
                if (lane >= (uint32_t)off) incl += o;
            }
            wave_sync();
            if (lane < (uint32_t)kNumClasses) cnt[lane] = incl - c;
            wave_sync();
#pragma unroll
            for (int i = 0; i < kSortPer; ++i) ent[cnt[v[i] >> kClassShift] + rk[i]] = v[i];
            wave_sync();
#pragma unroll 1
            for (int j = 0; j < kSortPer; ++j) one(ent[j * 64 + lane] & kIdMask);
            wave_sync();  // the next round rewrites the area
        }
    } else {
        const uint32_t idmask = B.nkey > 1 ? kIdMask : 0xffffffffu;
        if constexpr (FORM == kFormEdge) {
            // edge pairs: groups of 16 lanes read the list 16 entries (a
            // chunk) at a time, so that, the list being in rough id order, a
            // group reads 16 neighbouring 64-byte edge payloads (whole lines).
            // The list is cut into G stripes, one per group of the block;
            // chunk c is position c / G of stripe c % G, and each wavefront
            // takes the next four chunks from a counter in LDS.  Concurrent
            // groups then draw in separate stripes (16 neighbouring edges are
            // parallel and a few pixels apart: a whole wavefront of them would
            // crowd the same LDS banks), and a wavefront that finishes early
            // takes over chunks that a static share would have left to a
            // slow one (which holds up the whole block, as the tile's LDS
            // admits one block per CU).
            const uint32_t G = TPB / 16, g = threadIdx.x >> 4, q = threadIdx.x & 15u, gw = g & 3u;
            const uint32_t C = ((it.count + G - 1) / G + 15u) & ~15u;  // entries per stripe
            const uint32_t nchunk = G * (C / 16u);
            constexpr uint32_t kDone = 0xffffffffu, kNone = 0xfffffffeu;
            // this lane's entry of the wavefront's next chunk: kDone when the
            // chunks are used up (the same for the group's 16 lanes, and the
            // wavefront's first group is the last to run out, so its lane 0
            // is active for every call), kNone past the end of the list
            auto take = [&]() -> uint32_t {
                uint32_t c0 = 0u;
                if ((threadIdx.x & 63u) == 0u) c0 = atomicAdd(&s_next, 4u);
                const uint32_t c = (uint32_t)__builtin_amdgcn_readfirstlane((int)c0) + gw;
                if (c >= nchunk) return kDone;
                const uint32_t e = (c % G) * C + (c / G) * 16u + q;
                return e < it.count ? e : kNone;
            };
            // A pair's id and payload are two dependent loads; the next
            // pair's are issued before this one is drawn, so that they arrive
            // while it is (one wavefront per SIMD quarter has too little
            // other work to hide them otherwise).  (Two pairs ahead measured
            // slower: more registers in flight.)
            auto id_at = [&](uint32_t e) { return e < it.count ? pairs[it.first + e] : 0xffffffffu; };
            auto is_edge = [&](uint32_t id) { return id < B.ntet && id >= B.first_edge; };
            // a kink's two entries, at columns j and j + 1
            auto dep = [&](int row, int j, double v1, double v2) {
                const int x = cell(row, j);
                atomicAdd(&sA[x], v1);
                atomicAdd(&sA[x + 1], v2);
            };
            auto seam = [&](int row, double a, double b) {
                atomicAdd(&sSeam[row * nsc + sc], a);
                atomicAdd(&sSeam[(B.Th + row) * nsc + sc], b);
            };
            uint32_t e = take();
            uint32_t en = take();
            uint32_t id = id_at(e), idn = id_at(en);
            EdgePayload P{};
            if (is_edge(id)) P = ecoef[id - B.first_edge];
            // the first payload has arrived before the loop: the loop then
            // waits only for the loads it issued itself, at its end (without
            // this the wait before each pair's first use also takes the next
            // pair's loads)
            __builtin_amdgcn_s_waitcnt(0);
            // Seam lines are queued per wavefront (pair ids in LDS, after the
            // tile's seam arrays) and drawn 64 at a time with every lane busy:
            // about one pair in seven has one, and drawn as it comes each
            // held up its whole wavefront.  qn is the same in every active
            // lane; lane 0 is active for every round (its group runs out
            // last), so it holds the count after the loop.
            uint32_t *sQueue = reinterpret_cast<uint32_t *>(sA + tsize + nseam) + (threadIdx.x >> 6) * kSeamQueue;
            uint32_t qn = 0u;
            // queue entries first .. first + cnt - 1, taken in turn by the
            // active lanes (the edge job recomputed for its copy and rows)
            auto seam_entries = [&](uint32_t first, uint32_t cnt) {
                const uint64_t act = __builtin_amdgcn_read_exec();
                const uint32_t nact = (uint32_t)__builtin_popcountll(act);
                const uint32_t rank =
                    __builtin_amdgcn_mbcnt_hi((uint32_t)(act >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)act, 0u));
                for (uint32_t k = rank; k < cnt; k += nact) {
                    const uint32_t sid = sQueue[first + k];
                    const EdgePayload Q = ecoef[sid - B.first_edge];
                    uint32_t counted = 0u;  // (its kinks were counted when the pair was drawn)
                    const EdgeJob K = edge_job(Q, B, tx0, ty0, n, rows, counted);
                    edge_copy_seam(Q, sid - B.first_edge, B, tx0, n, K.kx, K.shift, K.ta - K.r0, K.r0,
                                   K.r0 + K.cnt - 1, Q.sl != 0.0 ? fast_rcp(Q.sl) : 0.0, seam, seam_range);
                }
            };
            while (e != kDone) {
                const uint32_t enn = take();
                const uint32_t idnn = id_at(enn);
                EdgePayload Pn{};
                if (is_edge(idn)) Pn = ecoef[idn - B.first_edge];
                if constexpr (COUNT) {
                    if (is_edge(id))
                        frags += (int32_t)edge_pair<COUNT>(P, id - B.first_edge, head[id].spare, B, tx0, ty0, n,
                                                           rows, dep, seam, seam_range, kinks);
                } else {
                    // the group's 16 edges one after another, each one's rows
                    // over the 16 lanes (consecutive rows: cells a row stride
                    // apart, in different banks), then the rest of a lane's own
                    // edge here: that copy's seam line, further copies (rare)
                    EdgeJob J{};
                    if (is_edge(id)) J = edge_job(P, B, tx0, ty0, n, rows, kinks);
                    const uint32_t pk = (uint32_t)J.cnt << 8;
                    const int row8 = (int)(uint32_t)(uintptr_t)(lds_f64 *)sA + J.ta * stride * 8;
                    const uint32_t p1 = (uint32_t)(row8 + (kPad + 1 - J.shift) * 8);
                    const uint32_t p2 = (uint32_t)(row8 + (kPad - 2) * 8);
                    const int qs8 = (int)q * stride * 8;
                    if (rows <= 32)
                        group_kinks<0, true>(J, pk, p1, p2, (int)q, qs8, (n + 2) * 8, stride * 8);
                    else
                        group_kinks<0, false>(J, pk, p1, p2, (int)q, qs8, (n + 2) * 8, stride * 8);
                    const uint64_t sm = __builtin_amdgcn_ballot_w64(J.seamed);
                    if (sm != 0ull) {
                        const uint32_t below =
                            __builtin_amdgcn_mbcnt_hi((uint32_t)(sm >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)sm, 0u));
                        if (J.seamed) sQueue[qn + below] = id;
                        qn += (uint32_t)__builtin_popcountll(sm);  // at most 63 + 64 < kSeamQueue
                        if (qn >= 64u) {
                            wave_sync();
                            seam_entries(0u, 64u);
                            // the rest (fewer than 64) to the front
                            const uint32_t rest = qn - 64u;
                            const uint64_t act = __builtin_amdgcn_read_exec();
                            const uint32_t nact = (uint32_t)__builtin_popcountll(act);
                            const uint32_t rank = __builtin_amdgcn_mbcnt_hi(
                                (uint32_t)(act >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)act, 0u));
                            wave_sync();
                            for (uint32_t k = rank; k < rest; k += nact) sQueue[k] = sQueue[64u + k];
                            wave_sync();
                            qn = rest;
                        }
                    }
                    if (J.more)
                        frags += (int32_t)edge_pair<false, true>(P, id - B.first_edge, 0u, B, tx0, ty0, n, rows, dep,
                                                                 seam, seam_range, kinks);
                }
                e = en;
                en = enn;
                id = idn;
                idn = idnn;
                P = Pn;
            }
            if constexpr (!COUNT) {
                qn = (uint32_t)__builtin_amdgcn_readfirstlane((int)qn);
                wave_sync();
                seam_entries(0u, qn);
            }
            const uint32_t g0 = g * C, g1 = min(it.count, g0 + C);
            // then the tetrahedra that kept their own records
            for (uint32_t e2 = g0 + q; e2 < g1; e2 += 16) {
                const uint32_t id2 = pairs[it.first + e2];
                if (id2 < B.first_edge) one(id2);
            }
        } else
        for (uint32_t e = e0; e < e1; e += kIdBurst) {
            // the next ids of the slice in one burst: one fetch of their cache
            // line serves kIdBurst pairs (read one at a time, microseconds
            // apart, the line is gone from L2 before its next use)
            uint32_t ids[kIdBurst];
#pragma unroll
            for (int i = 0; i < kIdBurst; ++i) ids[i] = e + i < e1 ? pairs[it.first + e + i] : 0xffffffffu;
            const int cnt = (int)min((uint32_t)kIdBurst, e1 - e);
            for (int i = 0; i < cnt; ++i) {
                const uint32_t id = ids[0] & idmask;
#pragma unroll
                for (int j = 0; j + 1 < kIdBurst; ++j) ids[j] = ids[j + 1];
                one(id);
            }
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < rows * B.Tw; i += TPB) {
        const int r = i / B.Tw, c = i - r * B.Tw;
        const double v = sA[cell(r, c)];
        if (c < n && v != 0.0) unsafeAtomicAdd(&acc[(int64_t)(ty0 + r) * B.W + tx0 + c], v);
    }
    // the seam lines: a at column 0 and b - a at column 1 of the second
    // differences; the range updates first summed over their copies (into
    // copy 0), then over the rows up to each row
    if (nsc) {
        for (int i = threadIdx.x; i < 3 * rows; i += TPB) {
            const int arr = i / rows, q = i - arr * rows;
            double *p = &sDiff[arr * dstride + q * nsc];
            double t = 0.0;
            for (int c = 0; c < nsc; ++c) t += p[c];
            p[0] = t;
        }
        __syncthreads();
        for (int r = threadIdx.x; r < rows; r += TPB) {
            double a = 0.0, b = 0.0, pa = 0.0, pb = 0.0, pg = 0.0;
            for (int c = 0; c < nsc; ++c) {
                a += sSeam[r * nsc + c];
                b += sSeam[(B.Th + r) * nsc + c];
            }
            for (int q = 0; q <= r; ++q) {
                pa += sDiff[q * nsc];
                pb += sDiff[dstride + q * nsc];
                pg += sDiff[2 * dstride + q * nsc];
            }
            a += pa + pb * (double)r;
            b += pg;
            if (a != 0.0) unsafeAtomicAdd(&acc[(int64_t)(ty0 + r) * B.W], a);
            if (B.W > 1 && b - a != 0.0) unsafeAtomicAdd(&acc[(int64_t)(ty0 + r) * B.W + 1], b - a);
        }
    }
    const unsigned long long f = wave_sum((unsigned long long)frags);
    const unsigned long long sp = wave_sum((unsigned long long)spans);
    const unsigned long long kk = wave_sum((unsigned long long)kinks);
    if ((threadIdx.x & 63) == 0) {
        if (f) atomicAdd(&counters->fragments, f);
        if (sp) atomicAdd(&counters->spans, sp);
        if (kk) atomicAdd(&counters->kinks, kk);
    }
}

template <int FORM, bool COUNT = true>
static void launch_raster_form(const RecHead *head, const Payload *coef, const EdgePayload *ecoef,
                               const uint32_t *pairs,
                               const WorkItem *items, uint64_t max_items, const PlanOut *plan,
                               const BinParams &B, int sorted, int block, double *acc, DevCounters *counters,
                               hipStream_t stream, size_t lds) {
    switch (block) {
        case 256:
            hipLaunchKernelGGL((k_raster<256, FORM, COUNT>), dim3((unsigned)max_items), dim3(256), lds, stream, head,
                               coef, ecoef, pairs, items, plan, B, sorted, acc, counters);
            break;
        case 512:
            hipLaunchKernelGGL((k_raster<512, FORM, COUNT>), dim3((unsigned)max_items), dim3(512), lds, stream, head,
                               coef, ecoef, pairs, items, plan, B, sorted, acc, counters);
            break;
        default:
            hipLaunchKernelGGL((k_raster<1024, FORM, COUNT>), dim3((unsigned)max_items), dim3(1024), lds, stream,
                               head, coef, ecoef, pairs, items, plan, B, sorted, acc, counters);
    }
}

hipError_t launch_raster(const RecHead *head, const Payload *coef, const EdgePayload *ecoef, const uint32_t *pairs,
                         const WorkItem *items, uint64_t max_items, const PlanOut *plan,
                         const BinParams &B, int block, bool count, double *acc, DevCounters *counters,
                         hipStream_t stream) {
    if (max_items == 0) return hipSuccess;
    if (block != 256 && block != 512 && block != 1024) return hipErrorInvalidValue;
    // the tile's accumulator, its seam lines (as many copies per row as fit,
    // up to 16), and beside them (when they fit) the wavefronts' class sorts
    BinParams Bl = B;
    const bool edge_form = B.form != kFormFace && B.form != kFormSplat && B.form != kFormPersp && B.edges;
    const size_t acc_lds = sizeof(double) * (size_t)B.Th * tile_stride(B.Tw, B.Th, edge_form);
    const size_t row_seam = sizeof(double) * (2 * (size_t)B.Th + 3 * ((size_t)B.Th + 1));
    const size_t queue_lds = edge_form ? sizeof(uint32_t) * (size_t)(block / 64) * kSeamQueue : 0;
    const size_t room = kLdsBytes > acc_lds + queue_lds ? kLdsBytes - acc_lds - queue_lds : 0;
    Bl.seam_copies = B.seam ? (int)std::min<size_t>(16, std::max<size_t>(1, room / row_seam)) : 0;
    const size_t tile_lds = acc_lds + row_seam * (size_t)Bl.seam_copies + queue_lds;
    if (tile_lds > kLdsBytes) return hipErrorInvalidValue;  // (tiles of at most 16384 cells fit)
    const size_t sort_lds = sizeof(uint32_t) * (size_t)(block / 64) * kSortWords;
    const int sorted = B.nkey > 1 && tile_lds + sort_lds <= kLdsBytes ? 1 : 0;
    const size_t lds = tile_lds + (sorted ? sort_lds : 0);
    if (Bl.form == kFormFace)
        launch_raster_form<kFormFace>(head, coef, ecoef, pairs, items, max_items, plan, Bl, sorted, block, acc, counters,
                                      stream, lds);
    else if (B.form == kFormSplat)
        launch_raster_form<kFormSplat>(head, coef, ecoef, pairs, items, max_items, plan, Bl, sorted, block, acc, counters,
                                       stream, lds);
    else if (B.form == kFormPersp)
        launch_raster_form<kFormPersp>(head, coef, ecoef, pairs, items, max_items, plan, Bl, sorted, block, acc, counters,
                                       stream, lds);
    else if (B.edges && count)
        launch_raster_form<kFormEdge, true>(head, coef, ecoef, pairs, items, max_items, plan, Bl, sorted, block, acc,
                                            counters, stream, lds);
    else if (B.edges)
        launch_raster_form<kFormEdge, false>(head, coef, ecoef, pairs, items, max_items, plan, Bl, sorted, block, acc,
                                             counters, stream, lds);
    else
        launch_raster_form<kFormPyramid>(head, coef, ecoef, pairs, items, max_items, plan, Bl, sorted, block, acc,
                                         counters, stream, lds);
    return hipGetLastError();
}

// ------------------------------------------------------- overflow raster
// When an image's (record, tile) pairs exceed the pair buffer, binning drops
// its lists and this kernel draws every record over the whole image instead:
// one thread per record, the image taken as row bands of kDirectRows rows
// (the crease form's row offsets are 8-bit), entries added into `acc` with
// L2 FP64 atomics.  Slow, but it needs no list, so the projection never has
// to read the pair count back before launching the raster.  Every other
// image returns at once.
constexpr int kDirectRows = 256;

template <int FORM>
__global__ void __launch_bounds__(256) k_raster_direct(LatticeParams L, ViewParams V,
                                                       const RecHead *__restrict__ head,
                                                       const Payload *__restrict__ coef,
                                                       const EdgePayload *__restrict__ ecoef,
                                                       const PlanOut *__restrict__ plan, unsigned long long cap,
                                                       BinParams B, double *__restrict__ acc,
                                                       DevCounters *__restrict__ counters) {
    const bool lists_dropped = plan->total_pairs > cap;
    const bool spilled = FORM == kFormEdge && plan->own > V.own_cap;
    if (!lists_dropped && !spilled) return;
    long long frags = 0;
    uint32_t spans = 0, kinks = 0;
    const int W = B.W;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, nth = (int64_t)gridDim.x * blockDim.x;
    // one record over the whole image, row band by row band
    auto draw = [&](const RecHead &h, const double *cf) {
        for (int ty0 = 0; ty0 < B.H; ty0 += kDirectRows) {
            const int rows = min(kDirectRows, B.H - ty0);
            auto dep = [&](int row, int j, double v) {
                if (j >= 0 && j < W) unsafeAtomicAdd(&acc[(int64_t)(ty0 + row) * W + j], v);
            };
            auto seam = [&](int row, double a, double b) {
                unsafeAtomicAdd(&acc[(int64_t)(ty0 + row) * W], a);
                if (W > 1) unsafeAtomicAdd(&acc[(int64_t)(ty0 + row) * W + 1], b - a);
            };
            if constexpr (FORM == kFormPersp)
                frags += persp_pair(h, cf, B, 0, ty0, W, rows, 0, 1, dep, spans, kinks);
            else
                frags += (int32_t)raster_record<FORM == kFormEdge ? kFormPyramid : FORM>(
                    h, cf, B, 0, ty0, W, rows, dep, seam, spans, kinks);
        }
    };
    if (lists_dropped)
        for (int64_t id = tid; id < (int64_t)B.ntet; id += nth) {
            const RecHead h = head[id];
            if (!(h.flags & REC_VALID)) continue;
            if constexpr (FORM == kFormEdge) {
                if ((uint32_t)id >= B.first_edge) {
                    for (int ty0 = 0; ty0 < B.H; ty0 += kDirectRows) {
                        const int rows = min(kDirectRows, B.H - ty0);
                        auto dep = [&](int row, int j, double v) {
                            if (j >= 0 && j < W) unsafeAtomicAdd(&acc[(int64_t)(ty0 + row) * W + j], v);
                        };
                        auto seam = [&](int row, double a, double b) {
                            unsafeAtomicAdd(&acc[(int64_t)(ty0 + row) * W], a);
                            if (W > 1) unsafeAtomicAdd(&acc[(int64_t)(ty0 + row) * W + 1], b - a);
                        };
                        frags += (int32_t)edge_pair(
                            ecoef[id - B.first_edge], (uint32_t)id - B.first_edge, h.spare, B, 0, ty0, W, rows,
                            [&](int row, int j, double v1, double v2) {
                                dep(row, j, v1);
                                dep(row, j + 1, v2);
                            },
                            seam,
                            [&](int lo, int hi, double alpha, double beta, double gamma) {
                                for (int r = lo; r <= hi; ++r) seam(r, alpha + beta * (double)r, gamma);
                            },
                            kinks);
                    }
                    continue;
                }
            }
            draw(h, coef[id].c);
        }
    if constexpr (FORM == kFormEdge) {
        // tetrahedra beyond the payload capacity: set up again (the same
        // record: the per-tetrahedron code of the edge form's setup without
        // its edge branch, which these did not take) and drawn
        if (spilled) {
            const int64_t nwords = (6 * L.ncubes + 31) / 32;
            for (int64_t w = tid; w < nwords; w += nth) {
                uint32_t bits = V.spill[w];
                while (bits) {
                    const int b = __builtin_ctz(bits);
                    bits &= bits - 1u;
                    const int64_t tet = 32 * w + b;
                    const int64_t cube = tet / 6;
                    const int t = (int)(tet - 6 * cube);
                    RecHead h{};
                    Payload P;
                    CubeCounts cc;
                    setup_cube<kFormPyramid, false>(
                        L, V, cube,
                        [&](int tt, const RecHead &R, const Payload &Q) {
                            if (tt == t) {
                                h = R;
                                P = Q;
                            }
                        },
                        cc);
                    if (h.flags & REC_VALID) draw(h, P.c);
                }
            }
        }
    }
    const unsigned long long f = wave_sum((unsigned long long)frags);
    const unsigned long long sp = wave_sum((unsigned long long)spans);
    const unsigned long long kk = wave_sum((unsigned long long)kinks);
    if ((threadIdx.x & 63) == 0) {
        if (f) atomicAdd(&counters->fragments, f);
        if (sp) atomicAdd(&counters->spans, sp);
        if (kk) atomicAdd(&counters->kinks, kk);
    }
}

hipError_t launch_raster_direct(const LatticeParams &L, const ViewParams &V, const RecHead *head,
                                const Payload *coef, const EdgePayload *ecoef, const PlanOut *plan,
                                unsigned long long cap, const BinParams &B, double *acc, DevCounters *counters,
                                hipStream_t stream) {
    // a small grid (threads stride over the records): the launch costs next
    // to nothing for the images that do not overflow
    const int64_t want = ((int64_t)B.ntet + 255) / 256;
    const dim3 grid((unsigned)(want < 2048 ? (want > 0 ? want : 1) : 2048)), block(256);
    switch (B.form) {
        case kFormFace:
            hipLaunchKernelGGL(k_raster_direct<kFormFace>, grid, block, 0, stream, L, V, head, coef, ecoef, plan, cap,
                               B, acc, counters);
            break;
        case kFormSplat:
            hipLaunchKernelGGL(k_raster_direct<kFormSplat>, grid, block, 0, stream, L, V, head, coef, ecoef, plan, cap,
                               B, acc, counters);
            break;
        case kFormPersp:
            hipLaunchKernelGGL(k_raster_direct<kFormPersp>, grid, block, 0, stream, L, V, head, coef, ecoef, plan, cap,
                               B, acc, counters);
            break;
        default:
            if (B.edges)
                hipLaunchKernelGGL(k_raster_direct<kFormEdge>, grid, block, 0, stream, L, V, head, coef, ecoef, plan,
                                   cap, B, acc, counters);
            else
                hipLaunchKernelGGL(k_raster_direct<kFormPyramid>, grid, block, 0, stream, L, V, head, coef, ecoef, plan,
                                   cap, B, acc, counters);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------- finalize
// One block per image row: f = running sum of the running sum of acc's row.
// Column densities are >= 0; a sum that rounding left a little below zero (a
// pixel no footprint covers, next to ones that do) is written as 0.
constexpr int kFinBlock = 256;

__device__ inline double block_exclusive_scan_f64(double v, double *sh, double &total) {
    // sh: kFinBlock / 64 + 1 entries; returns the exclusive prefix of v
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double incl = v;
    for (int off = 1; off < 64; off <<= 1) {
        const double o = __shfl_up(incl, off, 64);
        if (lane >= off) incl += o;
    }
    if (lane == 63) sh[wave] = incl;
    __syncthreads();
    double before = 0.0, all = 0.0;
    for (int w = 0; w < kFinBlock / 64; ++w) {
        if (w < wave) before += sh[w];
        all += sh[w];
    }
    __syncthreads();
    total = all;
    return before + incl - v;
}

__global__ void __launch_bounds__(kFinBlock) k_finalize(const double *__restrict__ acc, BinParams B,
                                                        float *__restrict__ image) {
    __shared__ double sh[kFinBlock / 64 + 1];
    const int y = blockIdx.x;
    const double *row = acc + (int64_t)y * B.W;
    float *out = image + (int64_t)y * B.W;
    if (B.direct) {
        // splats: the accumulator holds the values themselves
        for (int i = threadIdx.x; i < B.W; i += kFinBlock) out[i] = (float)fmax(row[i], 0.0);
        return;
    }
    const int per = (B.W + kFinBlock - 1) / kFinBlock;  // consecutive entries per thread
    const int i0 = threadIdx.x * per;
    // pass 1: d1 = running sum of A; the thread keeps its entries' d1 sum and
    // their d1-weighted contribution to the second running sum
    double s1 = 0.0;
    for (int k = 0; k < per; ++k)
        if (i0 + k < B.W) s1 += row[i0 + k];
    double tot;
    const double d1_in = block_exclusive_scan_f64(s1, sh, tot);  // d1 just before i0
    // pass 2: local second sum with the incoming d1
    double s2 = 0.0, d1 = d1_in;
    for (int k = 0; k < per; ++k)
        if (i0 + k < B.W) {
            d1 += row[i0 + k];
            s2 += d1;
        }
    const double f_in = block_exclusive_scan_f64(s2, sh, tot);  // f just before i0
    double f = f_in;
    d1 = d1_in;
    for (int k = 0; k < per; ++k)
        if (i0 + k < B.W) {
            d1 += row[i0 + k];
            f += d1;
            out[i0 + k] = (float)fmax(f, 0.0);
        }
}

hipError_t launch_finalize(const double *acc, const BinParams &B, float *image, hipStream_t stream) {
    hipLaunchKernelGGL(k_finalize, dim3((unsigned)B.H), dim3(kFinBlock), 0, stream, acc, B, image);
    return hipGetLastError();
}

// ------------------------------------------------- allocation-free scratch
// The workspace of tess_project_noalloc: one array per device, allocated when
// the library's code object is loaded on that device and held until the
// process ends.  Host code must not pass `scratch` itself to a kernel (on the
// host it names a stand-in, not device memory): scratch_buffer() returns its
// device address, taken once per device with that device current.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t scratch_buffer(void **ptr) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return hipSuccess;
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
