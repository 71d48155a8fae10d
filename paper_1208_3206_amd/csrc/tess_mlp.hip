// Refinement network kernels (gfx950): random Fourier features, a bf16 MFMA
// GEMM for the four 128-wide layers (forward and backward-data), a split-K
// MFMA GEMM for the weight gradients, the 128 -> 3 output layer, the mean
// squared error and Adam on FP32 master weights.
//
// Network: g = [sin 2 pi B q, cos 2 pi B q] (B integer, 64 x 3), then four
// times h = GELU(W h + b) (128 -> 128), then s = W5 h + b5 (128 -> 3).  The
// loss is the mean over samples of |s - target|^2.  bf16 operands, FP32
// accumulation, FP32 master weights.
#include "tess_mlp.h"
#include "tess_tet.h"  // the connectivity table (kTet)

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

namespace tess {
namespace mlp {

typedef __bf16 bf16;
typedef bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

// D(16x16) += A(16x32) * B(32x16) on one wavefront.  Lane l supplies
// A[l % 16][8 (l / 16) + j] and B[8 (l / 16) + j][l % 16] (j = 0..7) and
// receives D[4 (l / 16) + i][l % 16] (i = 0..3).
__device__ inline floatx4 mma16(bf16x8 a, bf16x8 b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ inline float gelu(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ inline float gelu_grad(float x) {
    const float cdf = 0.5f * (1.0f + erff(x * 0.70710678118654752f));
    const float pdf = 0.39894228040143268f * __expf(-0.5f * x * x);
    return cdf + x * pdf;
}

// ------------------------------------------------------------------ RFF
// X[n][f] = sin(2 pi B_f . q_n), X[n][64 + f] = cos(...), bf16.  B is integer,
// so sinpi/cospi of 2 B.q reduce exactly for dyadic q.
__global__ void k_rff(const float *__restrict__ q, int64_t n, const float *__restrict__ B,
                      bf16 *__restrict__ X) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * kFreq) return;
    const int64_t p = idx / kFreq;
    const int f = (int)(idx % kFreq);
    const float t = 2.0f * (B[3 * f] * q[3 * p] + B[3 * f + 1] * q[3 * p + 1] + B[3 * f + 2] * q[3 * p + 2]);
    X[p * kWidth + f] = (bf16)sinpif(t);
    X[p * kWidth + kFreq + f] = (bf16)cospif(t);
}

hipError_t launch_rff(const float *q, int64_t n, const float *B, bf16 *X, hipStream_t s) {
    const int64_t total = n * kFreq;
    hipLaunchKernelGGL(k_rff, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, q, n, B, X);
    return hipGetLastError();
}

// ------------------------------------------------------------ NT GEMM
// Y[n][o] = sum_i A[n][i] * M[o][i] for a 128 x 128 bf16 matrix M (row o
// contiguous), followed by an epilogue:
//   EPI_FWD : Z = Y + b (FP32, optional), H = GELU(Z) (bf16)
//   EPI_BWD : dZ = Y * GELU'(Zprev) (bf16)
// Each wavefront owns 16-row blocks (grid-stride); M sits in LDS.
enum { EPI_FWD = 0, EPI_BWD = 1 };

template <int EPI>
__global__ void __launch_bounds__(256) k_gemm_nt(const bf16 *__restrict__ A, int64_t n,
                                                 const bf16 *__restrict__ M,
                                                 const float *__restrict__ bias,
                                                 const float *__restrict__ Zin,
                                                 float *__restrict__ Zout, bf16 *__restrict__ Out) {
    constexpr int LDM = kWidth + 8;  // padded row (bf16 elements)
    __shared__ bf16 sM[kWidth * LDM];
    for (int e = threadIdx.x; e < kWidth * kWidth / 8; e += blockDim.x) {
        const int r = e / (kWidth / 8), c8 = e % (kWidth / 8);
        *(bf16x8 *)&sM[r * LDM + c8 * 8] = *(const bf16x8 *)&M[r * kWidth + c8 * 8];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int lr = lane & 15, lk = (lane >> 4) * 8;  // operand row/col and k offset
    const int64_t nblk = (n + 15) / 16;
    for (int64_t blk = (int64_t)blockIdx.x * 4 + wave; blk < nblk; blk += (int64_t)gridDim.x * 4) {
        const int64_t row0 = blk * 16;
        // A fragments for the four 32-wide k steps
        bf16x8 a[4];
        const int64_t ar = row0 + lr;
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            if (ar < n)
                a[ks] = *(const bf16x8 *)&A[ar * kWidth + ks * 32 + lk];
            else
                a[ks] = bf16x8{};
        }
#pragma unroll
        for (int ot = 0; ot < kWidth / 16; ++ot) {
            floatx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) {
                const bf16x8 b = *(const bf16x8 *)&sM[(ot * 16 + lr) * LDM + ks * 32 + lk];
                acc = mma16(a[ks], b, acc);
            }
            const int col = ot * 16 + lr;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int64_t row = row0 + (lane >> 4) * 4 + i;
                if (row >= n) continue;
                const int64_t o = row * kWidth + col;
                if (EPI == EPI_FWD) {
                    const float z = acc[i] + bias[col];
                    if (Zout) Zout[o] = z;
                    Out[o] = (bf16)gelu(z);
                } else {
                    Out[o] = (bf16)(acc[i] * gelu_grad(Zin[o]));
                }
            }
        }
    }
}

static int gemm_blocks(int64_t n) {
    const int64_t nblk = (n + 15) / 16;
    const int64_t want = (nblk + 3) / 4;
    return (int)(want < 4096 ? (want > 0 ? want : 1) : 4096);
}

hipError_t launch_layer_fwd(const bf16 *X, int64_t n, const bf16 *W, const float *b, float *Z,
                            bf16 *H, hipStream_t s) {
    hipLaunchKernelGGL(k_gemm_nt<EPI_FWD>, dim3(gemm_blocks(n)), dim3(256), 0, s, X, n, W, b,
                       (const float *)nullptr, Z, H);
    return hipGetLastError();
}

hipError_t launch_layer_bwd_data(const bf16 *dZ, int64_t n, const bf16 *WT, const float *Zprev,
                                 bf16 *dZprev, hipStream_t s) {
    hipLaunchKernelGGL(k_gemm_nt<EPI_BWD>, dim3(gemm_blocks(n)), dim3(256), 0, s, dZ, n, WT,
                       (const float *)nullptr, Zprev, (float *)nullptr, dZprev);
    return hipGetLastError();
}

// ------------------------------------------------------ weight gradient
// Partial dW[o][i] = sum over the slice's rows n of dZ[n][o] * H[n][i], and
// partial db[o] = sum dZ[n][o].  Slice rows are transposed into LDS so both
// MFMA operands are contiguous: A = dZ^T (o x n), B[n][i] = H[n][i] read as
// H^T rows.  Output: part[slice][128 * 128 + 128].
__global__ void __launch_bounds__(256) k_grad_w(const bf16 *__restrict__ dZ,
                                                const bf16 *__restrict__ H, int64_t n,
                                                float *__restrict__ part) {
    constexpr int LD = kSlice + 8;
    __shared__ bf16 sZT[kWidth * LD];
    __shared__ bf16 sHT[kWidth * LD];
    const int64_t r0 = (int64_t)blockIdx.x * kSlice;
    for (int e = threadIdx.x; e < kSlice * kWidth; e += blockDim.x) {
        const int r = e / kWidth, c = e % kWidth;
        const int64_t g = r0 + r;
        const bf16 z = g < n ? dZ[g * kWidth + c] : (bf16)0.0f;
        const bf16 h = g < n ? H[g * kWidth + c] : (bf16)0.0f;
        sZT[c * LD + r] = z;
        sHT[c * LD + r] = h;
    }
    __syncthreads();
    float *out = part + (size_t)blockIdx.x * (kWidth * kWidth + kWidth);
    if (threadIdx.x < kWidth) {
        float s = 0.f;
        for (int r = 0; r < kSlice; ++r) s += (float)sZT[threadIdx.x * LD + r];
        out[kWidth * kWidth + threadIdx.x] = s;
    }
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int lr = lane & 15, lk = (lane >> 4) * 8;
    // 64 output tiles (8 x 8 of 16 x 16); wave w takes tile rows 2w, 2w+1
#pragma unroll 1
    for (int tt = 0; tt < 16; ++tt) {
        const int to = wave * 2 + tt / 8, ti = tt % 8;
        floatx4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < kSlice / 32; ++ks) {
            const bf16x8 a = *(const bf16x8 *)&sZT[(to * 16 + lr) * LD + ks * 32 + lk];
            const bf16x8 b = *(const bf16x8 *)&sHT[(ti * 16 + lr) * LD + ks * 32 + lk];
            acc = mma16(a, b, acc);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int o = to * 16 + (lane >> 4) * 4 + i, c = ti * 16 + lr;
            out[o * kWidth + c] = acc[i];
        }
    }
}

hipError_t launch_grad_w(const bf16 *dZ, const bf16 *H, int64_t n, float *part, hipStream_t s) {
    const int64_t slices = (n + kSlice - 1) / kSlice;
    hipLaunchKernelGGL(k_grad_w, dim3((unsigned)slices), dim3(256), 0, s, dZ, H, n, part);
    return hipGetLastError();
}

// Deterministic sum over slices: out[e] = sum_s part[s][e].
__global__ void k_reduce_slices(const float *__restrict__ part, int64_t slices, int64_t stride,
                                int64_t count, float *__restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count) return;
    float s = 0.f;
    for (int64_t k = 0; k < slices; ++k) s += part[k * stride + e];
    out[e] = s;
}

hipError_t launch_reduce(const float *part, int64_t slices, int64_t stride, int64_t count, float *out,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_reduce_slices, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, part,
                       slices, stride, count, out);
    return hipGetLastError();
}

// ------------------------------------------------------- output layer
// pred[n][c] = sum_i H4[n][i] W5[c][i] + b5[c]; one thread per sample.
__global__ void k_out_fwd(const bf16 *__restrict__ H, int64_t n, const float *__restrict__ W5,
                          const float *__restrict__ b5, float *__restrict__ pred) {
    __shared__ float sW[3 * kWidth + 3];
    for (int e = threadIdx.x; e < 3 * kWidth; e += blockDim.x) sW[e] = (float)(bf16)W5[e];
    if (threadIdx.x < 3) sW[3 * kWidth + threadIdx.x] = b5[threadIdx.x];
    __syncthreads();
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    float a0 = 0.f, a1 = 0.f, a2 = 0.f;
    for (int i = 0; i < kWidth; i += 8) {
        const bf16x8 h = *(const bf16x8 *)&H[p * kWidth + i];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const float x = (float)h[j];
            a0 += x * sW[i + j];
            a1 += x * sW[kWidth + i + j];
            a2 += x * sW[2 * kWidth + i + j];
        }
    }
    pred[3 * p] = a0 + sW[3 * kWidth];
    pred[3 * p + 1] = a1 + sW[3 * kWidth + 1];
    pred[3 * p + 2] = a2 + sW[3 * kWidth + 2];
}

hipError_t launch_out_fwd(const bf16 *H, int64_t n, const float *W5, const float *b5, float *pred,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_out_fwd, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, H, n, W5, b5,
                       pred);
    return hipGetLastError();
}

// Loss terms and the output-layer backward, per block of 256 samples:
//   d = 2 (pred - target) / n,  dZ4[p][i] = (sum_c d[c] W5[c][i]) GELU'(Z4[p][i]),
//   part[blk] = {sum |pred - target|^2, dW5 partial (3 x 128), db5 partial (3)}.
constexpr int kOutBlk = 256;
__global__ void __launch_bounds__(kOutBlk) k_out_bwd(const float *__restrict__ pred,
                                                     const float *__restrict__ target, int64_t n,
                                                     const bf16 *__restrict__ H, const float *__restrict__ Z,
                                                     const float *__restrict__ W5,
                                                     bf16 *__restrict__ dZ, float *__restrict__ part) {
    __shared__ float sW[3 * kWidth];
    __shared__ float sd[kOutBlk * 3];
    __shared__ float sl[kOutBlk];
    for (int e = threadIdx.x; e < 3 * kWidth; e += blockDim.x) sW[e] = (float)(bf16)W5[e];
    const int64_t p = (int64_t)blockIdx.x * kOutBlk + threadIdx.x;
    float d0 = 0.f, d1 = 0.f, d2 = 0.f, l = 0.f;
    if (p < n) {
        const float e0 = pred[3 * p] - target[3 * p];
        const float e1 = pred[3 * p + 1] - target[3 * p + 1];
        const float e2 = pred[3 * p + 2] - target[3 * p + 2];
        l = e0 * e0 + e1 * e1 + e2 * e2;
        const float sc = 2.0f / (float)n;
        d0 = sc * e0; d1 = sc * e1; d2 = sc * e2;
    }
    sd[3 * threadIdx.x] = d0;
    sd[3 * threadIdx.x + 1] = d1;
    sd[3 * threadIdx.x + 2] = d2;
    sl[threadIdx.x] = l;
    __syncthreads();
    if (p < n) {
        for (int i = 0; i < kWidth; ++i) {
            const float g = d0 * sW[i] + d1 * sW[kWidth + i] + d2 * sW[2 * kWidth + i];
            dZ[p * kWidth + i] = (bf16)(g * gelu_grad(Z[p * kWidth + i]));
        }
    }
    // partial dW5[c][i] = sum over the block's samples of d[c] H[p][i]
    float *out = part + (size_t)blockIdx.x * kOutPart;
    const int64_t p0 = (int64_t)blockIdx.x * kOutBlk;
    for (int e = threadIdx.x; e < 3 * kWidth; e += blockDim.x) {
        const int c = e / kWidth, i = e % kWidth;
        float s = 0.f;
        for (int r = 0; r < kOutBlk; ++r) {
            if (p0 + r >= n) break;
            s += sd[3 * r + c] * (float)H[(p0 + r) * kWidth + i];
        }
        out[1 + e] = s;
    }
    if (threadIdx.x < 3) {
        float s = 0.f;
        for (int r = 0; r < kOutBlk; ++r) s += sd[3 * r + threadIdx.x];
        out[1 + 3 * kWidth + threadIdx.x] = s;
    }
    if (threadIdx.x == 0) {
        float s = 0.f;
        for (int r = 0; r < kOutBlk; ++r) s += sl[r];
        out[0] = s;
    }
}

hipError_t launch_out_bwd(const float *pred, const float *target, int64_t n, const bf16 *H,
                          const float *Z, const float *W5, bf16 *dZ, float *part, hipStream_t s) {
    hipLaunchKernelGGL(k_out_bwd, dim3((unsigned)((n + kOutBlk - 1) / kOutBlk)), dim3(kOutBlk), 0, s,
                       pred, target, n, H, Z, W5, dZ, part);
    return hipGetLastError();
}

int64_t out_blocks(int64_t n) { return (n + kOutBlk - 1) / kOutBlk; }

// ----------------------------------------------------------------- Adam
// In-place Adam on the FP32 master parameters (bias-corrected, step t >= 1).
// a1 = 1 - b1, a2 = 1 - b2 and the bias corrections c = 1 - b^t come from
// the host in FP64: in FP32 each difference cancels several digits (with
// b2 = 0.999, 1 - b2^t at small t keeps only about 4 of them)
__global__ void k_adam(float *__restrict__ w, float *__restrict__ m, float *__restrict__ v,
                       const float *__restrict__ g, int64_t count, float lr, float b1, float a1, float b2,
                       float a2, float eps, float c1, float c2) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count) return;
    const float gi = g[e];
    const float mi = b1 * m[e] + a1 * gi;
    const float vi = b2 * v[e] + a2 * gi * gi;
    m[e] = mi;
    v[e] = vi;
    w[e] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

hipError_t launch_adam(float *w, float *m, float *v, const float *g, int64_t count, double lr, double b1,
                       double b2, double eps, int t, hipStream_t s) {
    const double c1 = 1.0 - std::pow(b1, (double)t), c2 = 1.0 - std::pow(b2, (double)t);
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, w, m, v, g, count,
                       (float)lr, (float)b1, (float)(1.0 - b1), (float)b2, (float)(1.0 - b2), (float)eps,
                       (float)c1, (float)c2);
    return hipGetLastError();
}

// ------------------------------------------------------ fused inference
// The whole forward pass of one 16-sample tile on one wavefront, for
// inference: the features, the four hidden layers and the output layer stay
// in registers.  Each layer is computed transposed, D = W H^T (the weights
// as the MFMA's A operand, the activations as its B operand), so that after
// a layer the lane holding sample r = l % 16 has outputs o = 16 ot + 4 q + i
// (q = l / 16, i < 4, ot < 8): exactly the B operand of the next layer if
// that layer takes its input columns in the order k = 32 ks + 8 q + j <->
// input feature perm(k) = 16 (2 ks + j / 4) + 4 q + j % 4.  The weights are
// staged in LDS in that order, one 16-byte A fragment per lane per (layer,
// ot, ks); the first layer takes the features in their natural order, which
// the lanes compute for themselves.
constexpr int kInferWaves = 8;            // 512 threads; the staged weights admit one block per CU
constexpr int kFragsHidden = kDepth * 8 * 4 * 64;  // 16-byte fragments of the four hidden layers
constexpr int kFragsOut = 4 * 64;         // of the output layer (3 of its 16 rows are real)

__device__ __host__ inline int infer_perm(int k) {
    const int ks = k >> 5, q = (k >> 3) & 3, j = k & 7;
    return 16 * (2 * ks + (j >> 2)) + 4 * q + (j & 3);
}

__global__ void __launch_bounds__(64 * kInferWaves) k_mlp_infer(const float *__restrict__ q, int64_t n,
                                                                const float *__restrict__ B,
                                                                const float *__restrict__ master,
                                                                float *__restrict__ pred) {
    extern __shared__ bf16x8 sFrag[];                 // hidden, then output fragments
    __shared__ float sBias[kDepth * kWidth + 4];
    __shared__ float sB[3 * kFreq];
    // stage: fragment f of (layer, ot, ks, lane) holds W[o][perm or natural k .. +7]
    for (int f = threadIdx.x; f < kFragsHidden + kFragsOut; f += blockDim.x) {
        const int lane = f & 63, ks = (f >> 6) & 3;
        const bool out = f >= kFragsHidden;
        const int ot = out ? 0 : (f >> 8) & 7, l = out ? kDepth : f >> 11;
        const int o = 16 * ot + (lane & 15);
        bf16x8 v;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int k = 32 * ks + 8 * (lane >> 4) + j;
            const int kin = l == 0 ? k : infer_perm(k);
            float w = 0.f;
            if (!out)
                w = master[param_offset_W(l) + (int64_t)o * kWidth + kin];
            else if (o < 3)
                w = master[kOffW5 + (int64_t)o * kWidth + kin];
            v[j] = (bf16)w;
        }
        sFrag[f] = v;
    }
    for (int e = threadIdx.x; e < kDepth * kWidth; e += blockDim.x)
        sBias[e] = master[param_offset_b(e / kWidth) + e % kWidth];
    if (threadIdx.x < 3) sBias[kDepth * kWidth + threadIdx.x] = master[kOffB5 + threadIdx.x];
    for (int e = threadIdx.x; e < 3 * kFreq; e += blockDim.x) sB[e] = B[e];
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, lq = lane >> 4, lr = lane & 15;
    const int64_t ntile = (n + 15) / 16;
    for (int64_t tile = (int64_t)blockIdx.x * kInferWaves + wave; tile < ntile;
         tile += (int64_t)gridDim.x * kInferWaves) {
        const int64_t row = tile * 16 + lr;
        const bool live = row < n;
        // features of sample `row`, k = 32 ks + 8 q + j (natural order: sin
        // of frequency k for k < 64, cos of frequency k - 64 above)
        // (columns 64 apart are the sine and cosine of one frequency: k and
        // k + 64 sit in blocks ks and ks + 2 of the same lane)
        bf16x8 h[4];
        {
            const float q0 = live ? q[3 * row] : 0.f, q1 = live ? q[3 * row + 1] : 0.f,
                        q2 = live ? q[3 * row + 2] : 0.f;
#pragma unroll
            for (int ks = 0; ks < 2; ++ks)
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int f = 32 * ks + 8 * lq + j;
                    const float t = 2.0f * (sB[3 * f] * q0 + sB[3 * f + 1] * q1 + sB[3 * f + 2] * q2);
                    float sv, cv;
                    sincospif(t, &sv, &cv);
                    h[ks][j] = (bf16)sv;
                    h[ks + 2][j] = (bf16)cv;
                }
        }
#pragma unroll 1
        for (int l = 0; l < kDepth; ++l) {
            floatx4 acc[8];
#pragma unroll
            for (int ot = 0; ot < 8; ++ot) {
                acc[ot] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int ks = 0; ks < 4; ++ks)
                    acc[ot] = mma16(sFrag[((l * 8 + ot) * 4 + ks) * 64 + lane], h[ks], acc[ot]);
            }
            // bias, GELU, bf16: the next layer's operand (outputs 16 ot + 4 q + i
            // of this lane's sample, in the next layer's column order)
#pragma unroll
            for (int ks = 0; ks < 4; ++ks)
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int ot = 2 * ks + (j >> 2), i = j & 3;
                    const float z = acc[ot][i] + sBias[l * kWidth + 16 * ot + 4 * lq + i];
                    h[ks][j] = (bf16)gelu(z);
                }
        }
        floatx4 out = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) out = mma16(sFrag[kFragsHidden + ks * 64 + lane], h[ks], out);
        // lanes 0..15 hold outputs 0..3 of their sample (3 are real)
        if (lq == 0 && live) {
            pred[3 * row] = out[0] + sBias[kDepth * kWidth];
            pred[3 * row + 1] = out[1] + sBias[kDepth * kWidth + 1];
            pred[3 * row + 2] = out[2] + sBias[kDepth * kWidth + 2];
        }
    }
}

hipError_t launch_mlp_infer(const float *q, int64_t n, const float *B, const float *master, float *pred,
                            hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const int64_t tiles = (n + 15) / 16;
    const int64_t want = (tiles + kInferWaves - 1) / kInferWaves;
    const int blocks = (int)std::min<int64_t>(want, (int64_t)cus);
    const size_t lds = sizeof(bf16x8) * (size_t)(kFragsHidden + kFragsOut);
    hipLaunchKernelGGL(k_mlp_infer, dim3((unsigned)blocks), dim3(64 * kInferWaves), lds, s, q, n, B, master, pred);
    return hipGetLastError();
}

// bf16 copies of the four hidden weight matrices, row-major and transposed.
__global__ void k_cast_weights(const float *__restrict__ master, bf16 *__restrict__ Wb,
                               bf16 *__restrict__ WTb) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= kDepth * kWidth * kWidth) return;
    const int l = e / (kWidth * kWidth), r = (e / kWidth) % kWidth, c = e % kWidth;
    const float w = master[param_offset_W(l) + r * kWidth + c];
    Wb[e] = (bf16)w;
    WTb[l * kWidth * kWidth + c * kWidth + r] = (bf16)w;
}

hipError_t launch_cast_weights(const float *master, bf16 *Wb, bf16 *WTb, hipStream_t s) {
    const int total = kDepth * kWidth * kWidth;
    hipLaunchKernelGGL(k_cast_weights, dim3((total + 255) / 256), dim3(256), 0, s, master, Wb, WTb);
    return hipGetLastError();
}

}  // namespace mlp
}  // namespace tess

namespace tess {
namespace mlp {

// ------------------------------------------------------ refinement glue
// SplitMix64 (Steele, Lea & Flood 2014): counter-based 64-bit mixer.
__host__ __device__ inline uint64_t splitmix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ inline double min_image(double d, double L) { return d - L * ceil(d / L - 0.5); }

// Minibatch of `nb` coarse vertices drawn with replacement by a counter hash:
// q (unit torus) and the target displacement s = (x - q L) / L, minimal image.
__global__ void k_gather_batch(const float *__restrict__ x, const float *__restrict__ y,
                               const float *__restrict__ z, int d0, int d1, int d2, double L0,
                               double L1, double L2, uint64_t seed, uint64_t step, int64_t nb,
                               float *__restrict__ q, float *__restrict__ target) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nb) return;
    const int64_t n = (int64_t)d0 * d1 * d2;
    const int64_t id = (int64_t)(splitmix64(seed ^ (step * 0x100000001B3ull + (uint64_t)j)) % (uint64_t)n);
    const int i = (int)(id % d0), jj = (int)((id / d0) % d1), k = (int)(id / ((int64_t)d0 * d1));
    const double qu[3] = {(double)i / d0, (double)jj / d1, (double)k / d2};
    q[3 * j] = (float)qu[0];
    q[3 * j + 1] = (float)qu[1];
    q[3 * j + 2] = (float)qu[2];
    target[3 * j] = (float)(min_image((double)x[id] - qu[0] * L0, L0) / L0);
    target[3 * j + 1] = (float)(min_image((double)y[id] - qu[1] * L1, L1) / L1);
    target[3 * j + 2] = (float)(min_image((double)z[id] - qu[2] * L2, L2) / L2);
}

hipError_t launch_gather_batch(const float *x, const float *y, const float *z, const int dims[3],
                               const double box[3], uint64_t seed, uint64_t step, int64_t nb, float *q,
                               float *target, hipStream_t s) {
    hipLaunchKernelGGL(k_gather_batch, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, s, x, y, z,
                       dims[0], dims[1], dims[2], box[0], box[1], box[2], seed, step, nb, q, target);
    return hipGetLastError();
}

// Unit-torus coordinates of fine vertices first .. first + n - 1 (id order).
__global__ void k_fine_q(int64_t first, int64_t n, int f0, int f1, int f2, float *__restrict__ q) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int64_t id = first + j;
    q[3 * j] = (float)((double)(id % f0) / f0);
    q[3 * j + 1] = (float)((double)((id / f0) % f1) / f1);
    q[3 * j + 2] = (float)((double)(id / ((int64_t)f0 * f1)) / f2);
}

hipError_t launch_fine_q(int64_t first, int64_t n, const int fdims[3], float *q, hipStream_t s) {
    hipLaunchKernelGGL(k_fine_q, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, first, n, fdims[0],
                       fdims[1], fdims[2], q);
    return hipGetLastError();
}

__device__ inline float wrap_f32(double v, double L) {
    double w = v - L * floor(v / L);
    float f = (float)w;
    if (f >= (float)L) f -= (float)L;
    if (f < 0.f) f = 0.f;
    return f;
}

// Fine positions from the network: coarse vertices keep their data, the
// others get q L + s(q) L, wrapped into the box.
__global__ void k_place_mlp(const float *__restrict__ cx, const float *__restrict__ cy,
                            const float *__restrict__ cz, int d0, int d1, int r, int64_t first,
                            int64_t n, const float *__restrict__ q, const float *__restrict__ pred,
                            double L0, double L1, double L2, int f0, int f1, float *__restrict__ fx,
                            float *__restrict__ fy, float *__restrict__ fz) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int64_t id = first + j;
    const int I = (int)(id % f0), J = (int)((id / f0) % f1), K = (int)(id / ((int64_t)f0 * f1));
    if (I % r == 0 && J % r == 0 && K % r == 0) {
        const int64_t c = (int64_t)(I / r) + (int64_t)d0 * ((J / r) + (int64_t)d1 * (K / r));
        fx[id] = cx[c];
        fy[id] = cy[c];
        fz[id] = cz[c];
        return;
    }
    fx[id] = wrap_f32(((double)q[3 * j] + (double)pred[3 * j]) * L0, L0);
    fy[id] = wrap_f32(((double)q[3 * j + 1] + (double)pred[3 * j + 1]) * L1, L1);
    fz[id] = wrap_f32(((double)q[3 * j + 2] + (double)pred[3 * j + 2]) * L2, L2);
}

hipError_t launch_place_mlp(const float *cx, const float *cy, const float *cz, const int cdims[3], int r,
                            int64_t first, int64_t n, const float *q, const float *pred,
                            const double box[3], const int fdims[3], float *fx, float *fy, float *fz,
                            hipStream_t s) {
    hipLaunchKernelGGL(k_place_mlp, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, cx, cy, cz,
                       cdims[0], cdims[1], r, first, n, q, pred, box[0], box[1], box[2], fdims[0], fdims[1],
                       fx, fy, fz);
    return hipGetLastError();
}

// The tetrahedron of the unit cube's six-tetrahedron table (corner n = a +
// 2b + 4c at offset (a, b, c)) that contains point p, and p's barycentric
// coordinates in it (Cramer's rule); -1 if none does (not reached for points
// of the unit cube, which the six tetrahedra tile).
__device__ inline int unit_cube_tet(const double p[3], double lam[4]) {
    for (int t = 0; t < 6; ++t) {
        double R[4][3];
        for (int m = 0; m < 4; ++m) {
            const int c = kTet[t][m];
            R[m][0] = c & 1; R[m][1] = (c >> 1) & 1; R[m][2] = (c >> 2) & 1;
        }
        double M[3][3], rhs[3];
        for (int a = 0; a < 3; ++a) {
            for (int m = 0; m < 3; ++m) M[a][m] = R[m + 1][a] - R[0][a];
            rhs[a] = p[a] - R[0][a];
        }
        const double det = M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1]) -
                           M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0]) +
                           M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0]);
        for (int m = 0; m < 3; ++m) {
            double T[3][3];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) T[a][b] = (b == m) ? rhs[a] : M[a][b];
            lam[m + 1] = (T[0][0] * (T[1][1] * T[2][2] - T[1][2] * T[2][1]) -
                          T[0][1] * (T[1][0] * T[2][2] - T[1][2] * T[2][0]) +
                          T[0][2] * (T[1][0] * T[2][1] - T[1][1] * T[2][0])) / det;
        }
        lam[0] = 1.0 - lam[1] - lam[2] - lam[3];
        if (lam[0] < -1e-12 || lam[1] < -1e-12 || lam[2] < -1e-12 || lam[3] < -1e-12) continue;
        return t;
    }
    return -1;
}

__device__ inline int cube_corner(int t, int m) { return kTet[t][m]; }

// Fine positions by the affine map of the coarse tetrahedron that contains
// the vertex's Lagrangian point.
__global__ void k_place_linear(const float *__restrict__ cx, const float *__restrict__ cy,
                               const float *__restrict__ cz, int d0, int d1, int d2, int r,
                               double L0, double L1, double L2, int64_t nfine,
                               float *__restrict__ fx, float *__restrict__ fy, float *__restrict__ fz) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= nfine) return;
    const int f0 = d0 * r, f1 = d1 * r;
    const int I = (int)(id % f0), J = (int)((id / f0) % f1), K = (int)(id / ((int64_t)f0 * f1));
    const int i = I / r, j = J / r, k = K / r;
    const double p[3] = {(double)(I % r) / r, (double)(J % r) / r, (double)(K % r) / r};
    const double L[3] = {L0, L1, L2};
    // unwrapped corners of the coarse cube (periodic image nearest corner 0)
    double X[8][3];
    for (int c = 0; c < 8; ++c) {
        int ii = i + (c & 1), jj = j + ((c >> 1) & 1), kk = k + ((c >> 2) & 1);
        if (ii == d0) ii = 0;
        if (jj == d1) jj = 0;
        if (kk == d2) kk = 0;
        const int64_t cid = ii + (int64_t)d0 * (jj + (int64_t)d1 * kk);
        const double v[3] = {(double)cx[cid], (double)cy[cid], (double)cz[cid]};
        for (int a = 0; a < 3; ++a) {
            if (c == 0) {
                X[0][a] = v[a];
            } else {
                double e = v[a] - X[0][a];
                e -= L[a] * ceil(e / L[a] - 0.5);
                X[c][a] = X[0][a] + e;
            }
        }
    }
    double lam[4];
    const int t = unit_cube_tet(p, lam);
    double out[3] = {X[0][0], X[0][1], X[0][2]};
    if (t >= 0) {
        out[0] = out[1] = out[2] = 0.0;
        for (int m = 0; m < 4; ++m)
            for (int a = 0; a < 3; ++a) out[a] += lam[m] * X[cube_corner(t, m)][a];
    }
    fx[id] = wrap_f32(out[0], L0);
    fy[id] = wrap_f32(out[1], L1);
    fz[id] = wrap_f32(out[2], L2);
}

hipError_t launch_place_linear(const float *cx, const float *cy, const float *cz, const int cdims[3], int r,
                               const double box[3], float *fx, float *fy, float *fz, hipStream_t s) {
    const int64_t nfine = (int64_t)cdims[0] * cdims[1] * cdims[2] * r * r * r;
    hipLaunchKernelGGL(k_place_linear, dim3((unsigned)((nfine + 255) / 256)), dim3(256), 0, s, cx, cy, cz,
                       cdims[0], cdims[1], cdims[2], r, box[0], box[1], box[2], nfine, fx, fy, fz);
    return hipGetLastError();
}

// Residual of the network at coarse tracers first .. first+n-1 (q and pred
// of those tracers): x - (q + s(q)) L, as the periodic image in (-L/2, L/2].
__global__ void k_coarse_residual(const float *__restrict__ cx, const float *__restrict__ cy,
                                  const float *__restrict__ cz, int64_t first, int64_t n,
                                  const float *__restrict__ q, const float *__restrict__ pred, double L0,
                                  double L1, double L2, float *__restrict__ rx, float *__restrict__ ry,
                                  float *__restrict__ rz) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int64_t id = first + j;
    const double x[3] = {(double)cx[id], (double)cy[id], (double)cz[id]};
    const double L[3] = {L0, L1, L2};
    float *out[3] = {rx, ry, rz};
    for (int a = 0; a < 3; ++a) {
        double d = x[a] - ((double)q[3 * j + a] + (double)pred[3 * j + a]) * L[a];
        d -= L[a] * ceil(d / L[a] - 0.5);
        out[a][id] = (float)d;
    }
}

hipError_t launch_coarse_residual(const float *cx, const float *cy, const float *cz, int64_t first, int64_t n,
                                  const float *q, const float *pred, const double box[3], float *rx, float *ry,
                                  float *rz, hipStream_t s) {
    hipLaunchKernelGGL(k_coarse_residual, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, cx, cy, cz, first,
                       n, q, pred, box[0], box[1], box[2], rx, ry, rz);
    return hipGetLastError();
}

// Fine positions: network prediction plus the coarse residuals interpolated
// over the coarse tetrahedron that contains the vertex's Lagrangian point;
// coarse vertices keep their data exactly.
__global__ void k_place_hybrid(const float *__restrict__ cx, const float *__restrict__ cy,
                               const float *__restrict__ cz, const float *__restrict__ rx,
                               const float *__restrict__ ry, const float *__restrict__ rz, int d0, int d1,
                               int d2, int r, int64_t first, int64_t n, const float *__restrict__ q,
                               const float *__restrict__ pred, double L0, double L1, double L2,
                               float *__restrict__ fx, float *__restrict__ fy, float *__restrict__ fz) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int64_t id = first + j;
    const int f0 = d0 * r, f1 = d1 * r;
    const int I = (int)(id % f0), J = (int)((id / f0) % f1), K = (int)(id / ((int64_t)f0 * f1));
    const int i = I / r, jj0 = J / r, k = K / r;
    if (I % r == 0 && J % r == 0 && K % r == 0) {
        const int64_t c = (int64_t)i + (int64_t)d0 * (jj0 + (int64_t)d1 * k);
        fx[id] = cx[c];
        fy[id] = cy[c];
        fz[id] = cz[c];
        return;
    }
    const double p[3] = {(double)(I % r) / r, (double)(J % r) / r, (double)(K % r) / r};
    double lam[4];
    const int t = unit_cube_tet(p, lam);
    double res[3] = {0.0, 0.0, 0.0};
    for (int m = 0; m < 4 && t >= 0; ++m) {
        const int c = cube_corner(t, m);
        int ii = i + (c & 1), jj = jj0 + ((c >> 1) & 1), kk = k + ((c >> 2) & 1);
        if (ii == d0) ii = 0;
        if (jj == d1) jj = 0;
        if (kk == d2) kk = 0;
        const int64_t cid = ii + (int64_t)d0 * (jj + (int64_t)d1 * kk);
        res[0] += lam[m] * (double)rx[cid];
        res[1] += lam[m] * (double)ry[cid];
        res[2] += lam[m] * (double)rz[cid];
    }
    fx[id] = wrap_f32(((double)q[3 * j] + (double)pred[3 * j]) * L0 + res[0], L0);
    fy[id] = wrap_f32(((double)q[3 * j + 1] + (double)pred[3 * j + 1]) * L1 + res[1], L1);
    fz[id] = wrap_f32(((double)q[3 * j + 2] + (double)pred[3 * j + 2]) * L2 + res[2], L2);
}

hipError_t launch_place_hybrid(const float *cx, const float *cy, const float *cz, const float *rx,
                               const float *ry, const float *rz, const int cdims[3], int r, int64_t first,
                               int64_t n, const float *q, const float *pred, const double box[3], float *fx,
                               float *fy, float *fz, hipStream_t s) {
    hipLaunchKernelGGL(k_place_hybrid, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, cx, cy, cz, rx, ry, rz,
                       cdims[0], cdims[1], cdims[2], r, first, n, q, pred, box[0], box[1], box[2], fx, fy, fz);
    return hipGetLastError();
}

}  // namespace mlp
}  // namespace tess
