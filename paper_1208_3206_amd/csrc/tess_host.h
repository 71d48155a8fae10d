// Host-side pieces shared by the C ABI translation units.
#pragma once

#include "../../include/tess.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <cstdint>

// Lattice handle.
struct tess_lattice_s {
    tess_build_desc desc;
    const float *x, *y, *z;
    float *owned;  // one allocation holding x, y, z when the library owns them
    int device;
    int64_t n;
};

namespace tess {

// Sets the thread's error message and returns `st`.
tess_status fail(tess_status st, const char *fmt, ...);
tess_status ok();

#define TESS_HIP(call)                                                                   \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            return ::tess::fail(e_ == hipErrorOutOfMemory ? TESS_ENOMEM : TESS_EHIP,      \
                                "%s: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, __LINE__); \
    } while (0)

// Growable device buffer (elements of T).
template <typename T>
struct DevBuf {
    T *p = nullptr;
    size_t cap = 0;
    hipError_t ensure(size_t n) {
        if (n <= cap) return hipSuccess;
        if (p) {
            hipError_t e = hipFree(p);
            if (e != hipSuccess) return e;
            p = nullptr;
            cap = 0;
        }
        size_t want = std::max(n, (size_t)64);
        want += std::min(want / 8, headroom_max());  // headroom against small growth steps
        hipError_t e = hipMalloc((void **)&p, want * sizeof(T));
        if (e != hipSuccess) {
            p = nullptr;
            return e;
        }
        cap = want;
        return hipSuccess;
    }
    // bytes held after ensure(n)
    size_t bytes_after(size_t n) const {
        if (n <= cap) return cap * sizeof(T);
        const size_t want = std::max(n, (size_t)64);
        return (want + std::min(want / 8, headroom_max())) * sizeof(T);
    }
    // at most 64 MiB of headroom (an eighth of a multi-GB buffer would be GBs)
    static size_t headroom_max() { return ((size_t)64 << 20) / sizeof(T); }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        cap = 0;
    }
};

// Creates a lattice handle that owns `owned` (3 * n floats: x, y, z).
tess_lattice make_owned_lattice(const tess_build_desc &desc, float *owned, int device);

}  // namespace tess
