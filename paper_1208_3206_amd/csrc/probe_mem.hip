// Memory-system probe for the raster's two ceilings, a stand-alone program
// (not part of the library): the rate of FP64 (and 64-bit integer) atomic
// adds into LDS for the address patterns the raster produces, and the rate
// of 32-byte gathers from HBM at random positions.  Every LDS index is masked
// into the block's array and every gather index is reduced modulo the
// buffer's slot count.
//
// LDS patterns (kCells doubles per block, 16 wavefronts per block):
//   random   each lane a random cell (lanes drawing separate edges)
//   rows     16-lane groups at a random row, consecutive cells (16 lanes on
//            consecutive rows of one edge, rows a bank apart)
// with 64, 40 or 16 lanes of each wavefront active.
// Gathers: 32-byte reads at random 32-byte positions, two lanes on the two
// halves of a random 64-byte block, or four lanes on one random 128-byte line.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>

namespace {

constexpr int kCells = 4096;  // 32 KiB of doubles per block

__device__ __forceinline__ uint32_t mix(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7feb352dU;
    x ^= x >> 15;
    x *= 0x846ca68bU;
    x ^= x >> 16;
    return x;
}

template <typename T>
__global__ void __launch_bounds__(1024) k_lds_atomic(int iters, int active, int rows, T *out) {
    __shared__ T s[kCells];
    for (int i = threadIdx.x; i < kCells; i += blockDim.x) s[i] = (T)0;
    __syncthreads();
    const int lane = threadIdx.x & 63;
    uint32_t h = mix(blockIdx.x * 1024u + threadIdx.x + 12345u);
    if (lane < active) {
        for (int it = 0; it < iters; ++it) {
            const uint32_t idx = rows ? ((h >> 4) * 16u + (uint32_t)(lane & 15)) & (kCells - 1) : h & (kCells - 1);
            atomicAdd(&s[idx], (T)1);
            h = h * 1664525u + 1013904223u;
        }
    }
    __syncthreads();
    T acc = 0;
    for (int i = threadIdx.x; i < kCells; i += blockDim.x) acc += s[i];
    if (acc == (T)-1) out[0] = acc;  // never true: keeps the adds
}

// share: lanes per block of `share` slots that read the same random block
__global__ void __launch_bounds__(256) k_gather(const double4 *__restrict__ buf, uint64_t nslots, int iters, int share,
                                                double *out) {
    const uint32_t tid = blockIdx.x * 256u + threadIdx.x;
    uint32_t h = mix((tid / (uint32_t)share) * 2654435761u + 7u);
    double acc = 0.0;
    for (int it = 0; it < iters; ++it) {
        const uint64_t r = ((uint64_t)mix(h) << 20) ^ mix(h + 0x9e3779b9u);
        const uint64_t slot = (r % (nslots / (uint64_t)share)) * (uint64_t)share + (threadIdx.x % (uint32_t)share);
        const double4 v = buf[slot];
        acc += v.x + v.y + v.z + v.w;
        h = h * 1664525u + 1013904223u;
    }
    if (acc == -1.0) out[0] = acc;
}

#define CHECK(x)                                                                              \
    do {                                                                                      \
        const hipError_t e_ = (x);                                                            \
        if (e_ != hipSuccess) {                                                               \
            std::fprintf(stderr, "HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__); \
            return 1;                                                                         \
        }                                                                                     \
    } while (0)

template <typename T>
int lds_case(const char *name, int active, int rows, int cus, void *out) {
    const int iters = 4096, blocks = cus * 4;
    hipEvent_t a, b;
    CHECK(hipEventCreate(&a));
    CHECK(hipEventCreate(&b));
    k_lds_atomic<T><<<blocks, 1024>>>(64, active, rows, (T *)out);
    CHECK(hipGetLastError());
    CHECK(hipEventRecord(a));
    k_lds_atomic<T><<<blocks, 1024>>>(iters, active, rows, (T *)out);
    CHECK(hipGetLastError());
    CHECK(hipEventRecord(b));
    CHECK(hipEventSynchronize(b));
    float ms = 0.f;
    CHECK(hipEventElapsedTime(&ms, a, b));
    const double clocks = ms * 1e-3 * 2.4e9;
    const double lanes = (double)blocks * 16 * active * iters / cus;  // per CU
    const double insts = (double)blocks * 16 * iters / cus;
    std::printf("lds %-4s %-6s %2d lanes: %7.3f ms  %5.2f lane-adds/clk/CU  %5.1f clk per instruction\n", name,
                rows ? "rows" : "random", active, ms, lanes / clocks, clocks / insts);
    std::fflush(stdout);
    CHECK(hipEventDestroy(a));
    CHECK(hipEventDestroy(b));
    return 0;
}

}  // namespace

int main() {
    hipDeviceProp_t prop;
    CHECK(hipGetDeviceProperties(&prop, 0));
    const int cus = prop.multiProcessorCount;
    std::printf("%s, %d CUs (rates at 2.4 GHz)\n", prop.gcnArchName, cus);
    void *out = nullptr;
    CHECK(hipMalloc(&out, 64));
    for (int rows = 0; rows < 2; ++rows)
        for (int active : {64, 40, 16}) {
            if (lds_case<double>("f64", active, rows, cus, out)) return 1;
            if (lds_case<unsigned long long>("u64", active, rows, cus, out)) return 1;
        }
    const uint64_t bytes = 4ull << 30, nslots = bytes / 32;
    double4 *buf = nullptr;
    CHECK(hipMalloc(&buf, bytes));
    CHECK(hipMemset(buf, 0, bytes));
    for (int share : {1, 2, 4}) {
        const int iters = 256, blocks = cus * 64;
        hipEvent_t a, b;
        CHECK(hipEventCreate(&a));
        CHECK(hipEventCreate(&b));
        k_gather<<<blocks, 256>>>(buf, nslots, 8, share, (double *)out);
        CHECK(hipGetLastError());
        CHECK(hipEventRecord(a));
        k_gather<<<blocks, 256>>>(buf, nslots, iters, share, (double *)out);
        CHECK(hipGetLastError());
        CHECK(hipEventRecord(b));
        CHECK(hipEventSynchronize(b));
        float ms = 0.f;
        CHECK(hipEventElapsedTime(&ms, a, b));
        const double reads = (double)blocks * 256 * iters;
        const double blocks_read = reads / share;  // distinct 32 * share byte blocks
        std::printf("gather %3d-byte blocks: %7.3f ms  %6.1f G 32-byte reads/s  %5.1f G blocks/s = %4.2f TB/s of "
                    "128-byte lines\n",
                    32 * share, ms, reads / (ms * 1e-3) / 1e9, blocks_read / (ms * 1e-3) / 1e9,
                    blocks_read * 128 / (ms * 1e-3) / 1e12);
        std::fflush(stdout);
        CHECK(hipEventDestroy(a));
        CHECK(hipEventDestroy(b));
    }
    CHECK(hipFree(buf));
    CHECK(hipFree(out));
    return 0;
}
