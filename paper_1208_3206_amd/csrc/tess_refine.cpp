// C ABI of the learned refinement: training of the displacement network on a
// coarse lattice's own (q, x) pairs, inference on the r-fold sub-lattice and
// placement of the fine vertices; plus one forward/backward evaluation used to
// check the gradients.
#include "tess_host.h"
#include "tess_internal.h"
#include "tess_mlp.h"

#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

using namespace tess;
using namespace tess::mlp;

namespace {

// SplitMix64 on the host (counter-based; same published mixer as the device).
uint64_t mix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
double uniform01(uint64_t seed, uint64_t ctr) {
    return ((mix64(seed ^ mix64(ctr)) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}
double normal(uint64_t seed, uint64_t ctr) {  // Box-Muller
    const double u1 = uniform01(seed, 2 * ctr), u2 = uniform01(seed, 2 * ctr + 1);
    return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
}

// Device state of one network: parameters, optimiser moments, bf16 copies and
// the activations of one batch of up to `cap` samples.
struct Net {
    DevBuf<float> master, m, v, grad, B;
    DevBuf<__bf16> Wb, WTb;
    DevBuf<float> q, target, pred, part, outpart;
    DevBuf<__bf16> X, H[kDepth], dZ[2];
    DevBuf<float> Z[kDepth];
    int64_t cap = 0;
    ~Net() {
        master.release(); m.release(); v.release(); grad.release(); B.release();
        Wb.release(); WTb.release(); q.release(); target.release(); pred.release();
        part.release(); outpart.release(); X.release(); dZ[0].release(); dZ[1].release();
        for (int l = 0; l < kDepth; ++l) { H[l].release(); Z[l].release(); }
    }
};

// Training buffers (activations, gradient partials) for batches of up to
// `batch` samples when `train`; the sample and prediction buffers hold the
// larger of that and `infer_cap`, the chunk of the fused inference, which
// needs nothing else.
tess_status net_alloc(Net &net, int64_t batch, bool train, int64_t infer_cap = 0) {
    const int64_t cap = std::max(train ? batch : (int64_t)0, infer_cap);
    TESS_HIP(net.master.ensure(kParams));
    TESS_HIP(net.B.ensure(3 * kFreq));
    TESS_HIP(net.q.ensure((size_t)3 * cap));
    TESS_HIP(net.pred.ensure((size_t)3 * cap));
    if (train) {
        TESS_HIP(net.grad.ensure(kParams));
        TESS_HIP(net.m.ensure(kParams));
        TESS_HIP(net.v.ensure(kParams));
        TESS_HIP(net.Wb.ensure((size_t)kDepth * kWidth * kWidth));
        TESS_HIP(net.WTb.ensure((size_t)kDepth * kWidth * kWidth));
        TESS_HIP(net.target.ensure((size_t)3 * batch));
        TESS_HIP(net.X.ensure((size_t)kWidth * batch));
        for (int l = 0; l < kDepth; ++l) {
            TESS_HIP(net.H[l].ensure((size_t)kWidth * batch));
            TESS_HIP(net.Z[l].ensure((size_t)kWidth * batch));
        }
        TESS_HIP(net.dZ[0].ensure((size_t)kWidth * batch));
        TESS_HIP(net.dZ[1].ensure((size_t)kWidth * batch));
        const int64_t slices = (batch + kSlice - 1) / kSlice;
        TESS_HIP(net.part.ensure((size_t)slices * (kWidth * kWidth + kWidth)));
        TESS_HIP(net.outpart.ensure((size_t)out_blocks(batch) * kOutPart));
    }
    net.cap = cap;
    return TESS_OK;
}

// Forward pass over net.q[0 .. n); with `train` the pre-activations are kept.
tess_status net_forward(Net &net, int64_t n, bool train, hipStream_t s) {
    TESS_HIP(launch_rff(net.q.p, n, net.B.p, net.X.p, s));
    for (int l = 0; l < kDepth; ++l) {
        const __bf16 *in = l == 0 ? net.X.p : net.H[l - 1].p;
        TESS_HIP(launch_layer_fwd(in, n, net.Wb.p + (size_t)l * kWidth * kWidth,
                                  net.master.p + param_offset_b(l), train ? net.Z[l].p : nullptr,
                                  net.H[l].p, s));
    }
    TESS_HIP(launch_out_fwd(net.H[kDepth - 1].p, n, net.master.p + kOffW5, net.master.p + kOffB5,
                            net.pred.p, s));
    return TESS_OK;
}

// Backward pass after net_forward(train): fills net.grad; the summed squared
// error lands in net.grad's scratch tail read by the caller (see loss_sum).
tess_status net_backward(Net &net, int64_t n, float *loss_sum, hipStream_t s) {
    TESS_HIP(launch_out_bwd(net.pred.p, net.target.p, n, net.H[kDepth - 1].p, net.Z[kDepth - 1].p,
                            net.master.p + kOffW5, net.dZ[0].p, net.outpart.p, s));
    int cur = 0;
    const int64_t slices = (n + kSlice - 1) / kSlice;
    for (int l = kDepth - 1; l >= 0; --l) {
        const __bf16 *hin = l == 0 ? net.X.p : net.H[l - 1].p;
        TESS_HIP(launch_grad_w(net.dZ[cur].p, hin, n, net.part.p, s));
        TESS_HIP(launch_reduce(net.part.p, slices, kLayerParams, kLayerParams,
                               net.grad.p + param_offset_W(l), s));
        if (l > 0) {
            TESS_HIP(launch_layer_bwd_data(net.dZ[cur].p, n, net.WTb.p + (size_t)l * kWidth * kWidth,
                                           net.Z[l - 1].p, net.dZ[1 - cur].p, s));
            cur = 1 - cur;
        }
    }
    // output layer: [loss, dW5, db5] summed over blocks; dW5/db5 land in grad
    const int64_t ob = out_blocks(n);
    TESS_HIP(launch_reduce(net.outpart.p + 1, ob, kOutPart, kOutPart - 1, net.grad.p + kOffW5, s));
    if (loss_sum) TESS_HIP(launch_reduce(net.outpart.p, ob, kOutPart, 1, loss_sum, s));
    return TESS_OK;
}

void init_params(std::vector<float> &p, uint64_t seed) {
    p.assign(kParams, 0.f);
    uint64_t ctr = 0;
    auto fill = [&](int64_t off, int64_t count, int fan_in) {
        const double k = 1.0 / std::sqrt((double)fan_in);
        for (int64_t e = 0; e < count; ++e) p[off + e] = (float)(k * (2.0 * uniform01(seed, ctr++) - 1.0));
    };
    for (int l = 0; l < kDepth; ++l) {
        fill(param_offset_W(l), (int64_t)kWidth * kWidth, kWidth);
        fill(param_offset_b(l), kWidth, kWidth);
    }
    fill(kOffW5, 3 * kWidth, kWidth);
    fill(kOffB5, 3, kWidth);
}

tess_status check_rff(const float *B) {
    for (int e = 0; e < 3 * kFreq; ++e)
        if (!std::isfinite(B[e]) || B[e] != std::rint(B[e]) || std::fabs(B[e]) > 1e6f)
            return fail(TESS_EINVAL, "rff_B[%d] must be a finite integer value", e);
    return TESS_OK;
}

}  // namespace

extern "C" tess_status tess_refine_desc_default(tess_refine_desc *d) {
    if (!d) return fail(TESS_EINVAL, "desc is NULL");
    std::memset(d, 0, sizeof(*d));
    d->r = 4;
    d->mode = TESS_REFINE_MLP;
    d->rff_sigma = 8.0;
    d->steps = 10000;
    d->batch = 8192;
    d->lr0 = 1e-2;
    d->lr1 = 1e-5;
    d->seed = 2;
    return ok();
}

extern "C" tess_status tess_mlp_loss_grad(const float *params, const float *rff_B, const float *q,
                                          const float *target, int64_t n, double *loss, float *grad,
                                          float *pred, void *stream) {
    if (!params || !rff_B || !q || !target) return fail(TESS_EINVAL, "NULL argument");
    if (n < 1 || n > (int64_t)1 << 26) return fail(TESS_EINVAL, "n = %lld outside 1..2^26", (long long)n);
    tess_status st = check_rff(rff_B);
    if (st != TESS_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    Net net;
    st = net_alloc(net, n, true);
    if (st != TESS_OK) return st;
    TESS_HIP(hipMemcpyAsync(net.master.p, params, sizeof(float) * kParams, hipMemcpyHostToDevice, s));
    TESS_HIP(hipMemcpyAsync(net.B.p, rff_B, sizeof(float) * 3 * kFreq, hipMemcpyHostToDevice, s));
    TESS_HIP(hipMemcpyAsync(net.q.p, q, sizeof(float) * 3 * n, hipMemcpyDeviceToDevice, s));
    TESS_HIP(hipMemcpyAsync(net.target.p, target, sizeof(float) * 3 * n, hipMemcpyDeviceToDevice, s));
    TESS_HIP(launch_cast_weights(net.master.p, net.Wb.p, net.WTb.p, s));
    st = net_forward(net, n, true, s);
    if (st != TESS_OK) return st;
    float *dloss = net.m.p;  // scratch: one float
    st = net_backward(net, n, dloss, s);
    if (st != TESS_OK) return st;
    float lsum = 0.f;
    TESS_HIP(hipMemcpyAsync(&lsum, dloss, sizeof(float), hipMemcpyDeviceToHost, s));
    if (grad) TESS_HIP(hipMemcpyAsync(grad, net.grad.p, sizeof(float) * kParams, hipMemcpyDeviceToHost, s));
    if (pred) TESS_HIP(hipMemcpyAsync(pred, net.pred.p, sizeof(float) * 3 * n, hipMemcpyDeviceToDevice, s));
    TESS_HIP(hipStreamSynchronize(s));
    if (loss) *loss = (double)lsum / (double)n;
    return ok();
}

extern "C" tess_status tess_mlp_forward(const float *params, const float *rff_B, const float *q, int64_t n,
                                        float *pred, void *stream) {
    if (!params || !rff_B || !q || !pred) return fail(TESS_EINVAL, "NULL argument");
    if (n < 1 || n > (int64_t)1 << 30) return fail(TESS_EINVAL, "n = %lld outside 1..2^30", (long long)n);
    tess_status st = check_rff(rff_B);
    if (st != TESS_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    DevBuf<float> buf;  // params, then the frequencies
    TESS_HIP(buf.ensure((size_t)kParams + 3 * kFreq));
    TESS_HIP(hipMemcpyAsync(buf.p, params, sizeof(float) * kParams, hipMemcpyHostToDevice, s));
    TESS_HIP(hipMemcpyAsync(buf.p + kParams, rff_B, sizeof(float) * 3 * kFreq, hipMemcpyHostToDevice, s));
    const hipError_t e = launch_mlp_infer(q, n, buf.p + kParams, buf.p, pred, s);
    const hipError_t w = hipStreamSynchronize(s);
    buf.release();
    if (e != hipSuccess || w != hipSuccess)
        return fail(TESS_EHIP, "inference: %s", hipGetErrorString(e != hipSuccess ? e : w));
    return ok();
}

extern "C" tess_status tess_mlp_adam(float *params, float *m, float *v, const float *grad, int32_t step, double lr,
                                     double beta1, double beta2, double eps, void *stream) {
    if (!params || !m || !v || !grad) return fail(TESS_EINVAL, "NULL argument");
    if (step < 1) return fail(TESS_EINVAL, "step must be >= 1");
    if (!(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
        return fail(TESS_EINVAL, "need lr > 0, 0 <= beta1, beta2 < 1 and eps > 0");
    hipStream_t s = (hipStream_t)stream;
    DevBuf<float> buf;  // params, m, v, grad
    TESS_HIP(buf.ensure((size_t)4 * kParams));
    float *dp = buf.p, *dm = buf.p + kParams, *dv = buf.p + 2 * kParams, *dg = buf.p + 3 * kParams;
    auto run = [&]() -> tess_status {
        TESS_HIP(hipMemcpyAsync(dp, params, sizeof(float) * kParams, hipMemcpyHostToDevice, s));
        TESS_HIP(hipMemcpyAsync(dm, m, sizeof(float) * kParams, hipMemcpyHostToDevice, s));
        TESS_HIP(hipMemcpyAsync(dv, v, sizeof(float) * kParams, hipMemcpyHostToDevice, s));
        TESS_HIP(hipMemcpyAsync(dg, grad, sizeof(float) * kParams, hipMemcpyHostToDevice, s));
        TESS_HIP(launch_adam(dp, dm, dv, dg, kParams, lr, beta1, beta2, eps, step, s));
        TESS_HIP(hipMemcpyAsync(params, dp, sizeof(float) * kParams, hipMemcpyDeviceToHost, s));
        TESS_HIP(hipMemcpyAsync(m, dm, sizeof(float) * kParams, hipMemcpyDeviceToHost, s));
        TESS_HIP(hipMemcpyAsync(v, dv, sizeof(float) * kParams, hipMemcpyDeviceToHost, s));
        TESS_HIP(hipStreamSynchronize(s));
        return TESS_OK;
    };
    const tess_status st = run();
    buf.release();
    return st == TESS_OK ? ok() : st;
}

extern "C" tess_status tess_refine(tess_lattice coarse, const tess_refine_desc *d, tess_lattice *fine,
                                   tess_refine_report *report, void *stream) {
    if (!coarse || !d || !fine) return fail(TESS_EINVAL, "NULL argument");
    *fine = nullptr;
    if (!coarse->desc.periodic) return fail(TESS_ENOTSUP, "refinement needs a periodic lattice");
    if (d->r < 1 || d->r > 16) return fail(TESS_EINVAL, "r = %d outside 1..16", d->r);
    if (d->mode != TESS_REFINE_LINEAR && d->mode != TESS_REFINE_MLP && d->mode != TESS_REFINE_MLP_RAW)
        return fail(TESS_EINVAL, "mode must be TESS_REFINE_LINEAR, TESS_REFINE_MLP or TESS_REFINE_MLP_RAW");
    int cd[3], fd[3];
    int64_t nfine = 1;
    for (int a = 0; a < 3; ++a) {
        cd[a] = coarse->desc.dims[a];
        fd[a] = cd[a] * d->r;
        nfine *= fd[a];
    }
    if (nfine * 6 > ((int64_t)1 << 32) - 1) return fail(TESS_ECAPACITY, "fine lattice too large");
    if (d->mode != TESS_REFINE_LINEAR) {
        if (d->steps < 0 || (d->steps == 0 && !d->weights_in))
            return fail(TESS_EINVAL, "steps must be > 0, or 0 with weights_in");
        if (d->batch < 64 || d->batch > (1 << 22)) return fail(TESS_EINVAL, "batch outside 64..2^22");
        if (!(d->lr0 > 0) || !(d->lr1 >= 0) || !(d->rff_sigma > 0))
            return fail(TESS_EINVAL, "lr0 > 0, lr1 >= 0 and rff_sigma > 0 are required");
    }
    hipStream_t s = (hipStream_t)stream;
    int dev = 0;
    TESS_HIP(hipGetDevice(&dev));
    if (dev != coarse->device) return fail(TESS_EINVAL, "lattice lives on another device");
    float *owned = nullptr;
    TESS_HIP(hipMalloc((void **)&owned, sizeof(float) * 3 * (size_t)nfine));
    float *fx = owned, *fy = owned + nfine, *fz = owned + 2 * nfine;
    auto fail_free = [&](tess_status st) {
        (void)hipFree(owned);
        return st;
    };
    tess_refine_report rep;
    std::memset(&rep, 0, sizeof(rep));
    rep.fine_tracers = nfine;
    const double *box = coarse->desc.box;
    if (d->mode == TESS_REFINE_LINEAR) {
        auto t0 = std::chrono::steady_clock::now();
        if (launch_place_linear(coarse->x, coarse->y, coarse->z, cd, d->r, box, fx, fy, fz, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return fail_free(fail(TESS_EHIP, "linear placement failed"));
        rep.infer_ms = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - t0).count();
    } else {
        // ---------------------------------------------------------- train
        std::vector<float> B(3 * kFreq), params;
        if (d->rff_B) {
            std::memcpy(B.data(), d->rff_B, sizeof(float) * B.size());
            tess_status st = check_rff(B.data());
            if (st != TESS_OK) return fail_free(st);
        } else {
            for (int e = 0; e < 3 * kFreq; ++e) B[e] = (float)std::rint(d->rff_sigma * normal(d->seed ^ 0xB5ull, e));
        }
        if (d->weights_in) {
            params.assign(d->weights_in, d->weights_in + kParams);
        } else {
            init_params(params, d->seed);
        }
        Net net;
        const int64_t cap = (int64_t)1 << 20;  // inference chunk
        const bool train = d->steps > 0;
        tess_status st = net_alloc(net, d->batch, train, cap);
        if (st != TESS_OK) return fail_free(st);
        TESS_HIP(hipMemcpyAsync(net.master.p, params.data(), sizeof(float) * kParams, hipMemcpyHostToDevice, s));
        TESS_HIP(hipMemcpyAsync(net.B.p, B.data(), sizeof(float) * B.size(), hipMemcpyHostToDevice, s));
        float *dloss = nullptr;
        if (train) {
            TESS_HIP(hipMemsetAsync(net.m.p, 0, sizeof(float) * kParams, s));
            TESS_HIP(hipMemsetAsync(net.v.p, 0, sizeof(float) * kParams, s));
            TESS_HIP(launch_cast_weights(net.master.p, net.Wb.p, net.WTb.p, s));
            TESS_HIP(hipMalloc((void **)&dloss, sizeof(float)));
        }
        auto t0 = std::chrono::steady_clock::now();
        float lsum = 0.f;
        const int64_t nb = d->batch;
        for (int step = 1; step <= d->steps; ++step) {
            if (launch_gather_batch(coarse->x, coarse->y, coarse->z, cd, box, d->seed + 1, (uint64_t)step, nb,
                                    net.q.p, net.target.p, s) != hipSuccess)
                return fail_free(fail(TESS_EHIP, "batch gather failed"));
            st = net_forward(net, nb, true, s);
            if (st == TESS_OK) st = net_backward(net, nb, (step == 1 || step == d->steps) ? dloss : nullptr, s);
            if (st != TESS_OK) {
                (void)hipFree(dloss);
                return fail_free(st);
            }
            if (step == 1 || step == d->steps) {
                TESS_HIP(hipMemcpyAsync(&lsum, dloss, sizeof(float), hipMemcpyDeviceToHost, s));
                TESS_HIP(hipStreamSynchronize(s));
                if (step == 1) rep.loss_first = lsum / (double)nb;
                rep.loss_last = lsum / (double)nb;
            }
            const double c = 0.5 * (1.0 + std::cos(3.141592653589793 * (double)(step - 1) / std::max(1, d->steps - 1)));
            const double lr = d->lr1 + (d->lr0 - d->lr1) * c;
            TESS_HIP(launch_adam(net.master.p, net.m.p, net.v.p, net.grad.p, kParams, lr, 0.9, 0.999, 1e-8, step, s));
            TESS_HIP(launch_cast_weights(net.master.p, net.Wb.p, net.WTb.p, s));
        }
        TESS_HIP(hipStreamSynchronize(s));
        (void)hipFree(dloss);
        rep.train_ms = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - t0).count();
        if (d->weights_out)
            TESS_HIP(hipMemcpy(d->weights_out, net.master.p, sizeof(float) * kParams, hipMemcpyDeviceToHost));
        // ------------------------------------------------------ inference
        t0 = std::chrono::steady_clock::now();
        float *res = nullptr;  // residuals at the coarse tracers (x, y, z arrays)
        const int64_t ncoarse = (int64_t)cd[0] * cd[1] * cd[2];
        if (d->mode == TESS_REFINE_MLP) {
            TESS_HIP(hipMalloc((void **)&res, sizeof(float) * 3 * (size_t)ncoarse));
            for (int64_t first = 0; first < ncoarse; first += cap) {
                const int64_t n = std::min<int64_t>(cap, ncoarse - first);
                TESS_HIP(launch_fine_q(first, n, cd, net.q.p, s));
                st = launch_mlp_infer(net.q.p, n, net.B.p, net.master.p, net.pred.p, s) == hipSuccess
                         ? TESS_OK
                         : fail(TESS_EHIP, "inference failed");
                if (st == TESS_OK &&
                    launch_coarse_residual(coarse->x, coarse->y, coarse->z, first, n, net.q.p, net.pred.p, box,
                                           res, res + ncoarse, res + 2 * ncoarse, s) != hipSuccess)
                    st = fail(TESS_EHIP, "coarse residual failed");
                if (st != TESS_OK) {
                    (void)hipFree(res);
                    return fail_free(st);
                }
            }
        }
        for (int64_t first = 0; first < nfine; first += cap) {
            const int64_t n = std::min<int64_t>(cap, nfine - first);
            TESS_HIP(launch_fine_q(first, n, fd, net.q.p, s));
            st = launch_mlp_infer(net.q.p, n, net.B.p, net.master.p, net.pred.p, s) == hipSuccess
                     ? TESS_OK
                     : fail(TESS_EHIP, "inference failed");
            hipError_t e = hipSuccess;
            if (st == TESS_OK) {
                if (res)
                    e = launch_place_hybrid(coarse->x, coarse->y, coarse->z, res, res + ncoarse, res + 2 * ncoarse,
                                            cd, d->r, first, n, net.q.p, net.pred.p, box, fx, fy, fz, s);
                else
                    e = launch_place_mlp(coarse->x, coarse->y, coarse->z, cd, d->r, first, n, net.q.p,
                                         net.pred.p, box, fd, fx, fy, fz, s);
            }
            if (st != TESS_OK || e != hipSuccess) {
                if (res) (void)hipFree(res);
                return fail_free(st != TESS_OK ? st : fail(TESS_EHIP, "placement failed"));
            }
        }
        TESS_HIP(hipStreamSynchronize(s));
        if (res) (void)hipFree(res);
        rep.infer_ms = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    {  // every placed position finite (a diverged network is reported, not rendered)
        unsigned long long *flag = nullptr, bad = 0, none = ~0ull;
        if (hipMalloc((void **)&flag, sizeof(*flag)) != hipSuccess) return fail_free(fail(TESS_ENOMEM, "flag"));
        const bool okc = hipMemcpyAsync(flag, &none, sizeof(none), hipMemcpyHostToDevice, s) == hipSuccess &&
                         launch_check_finite(fx, fy, fz, nfine, flag, s) == hipSuccess &&
                         hipMemcpyAsync(&bad, flag, sizeof(bad), hipMemcpyDeviceToHost, s) == hipSuccess &&
                         hipStreamSynchronize(s) == hipSuccess;
        (void)hipFree(flag);
        if (!okc) return fail_free(fail(TESS_EHIP, "finite check of the refined positions failed"));
        if (bad != ~0ull)
            return fail_free(fail(TESS_ERANGE, "refined position of tracer %llu is not finite", bad));
    }
    tess_build_desc fdesc = coarse->desc;
    for (int a = 0; a < 3; ++a) fdesc.dims[a] = fd[a];
    fdesc.copy_positions = 1;
    *fine = make_owned_lattice(fdesc, owned, dev);
    if (report) *report = rep;
    return ok();
}
