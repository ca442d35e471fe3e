// The FP64 direct sum of eq. StoStre for callers that cannot allocate device memory
// (work under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
//
// stk_direct allocates a buffer for the partial velocities of every (target, source
// chunk) per call.  This variant keeps them in `scratch`, a fixed array that every device
// the library runs on holds until the process ends, and runs the same kernels with the
// same source chunks, so its results equal stk_direct's bit for bit.  When the partials
// of all m targets do not fit, the targets go through in slices (the chunking is still
// that of the whole call).  Every call on a device shares that device's array: calls
// that overlap on one device race and must be ordered by the caller (one stream, or
// events).  Nothing in the array needs clearing: each slice writes every partial it
// later reads.
#include <mutex>
#include <vector>

#include "stk_internal.hpp"

static __device__ __align__(256) double scratch[STK_DIRECT_NOALLOC_SCRATCH_BYTES / sizeof(double)];

namespace stk {

namespace {

// Device address of `scratch` on device `dev` (which is current): looked up once per
// device.  In host code `scratch` names a host-side stand-in, never the device memory.
double *scratch_on(int dev) {
    static std::mutex mu;
    static std::vector<double *> *addr = new std::vector<double *>();
    std::lock_guard<std::mutex> lk(mu);
    if (size_t(dev) >= addr->size()) addr->resize(size_t(dev) + 1, nullptr);
    double *&a = (*addr)[size_t(dev)];
    if (!a) {
        void *p = nullptr;
        STK_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        require(p != nullptr, "hipGetSymbolAddress returned NULL for the direct-sum scratch array");
        a = static_cast<double *>(p);
    }
    return a;
}

}  // namespace

int64_t direct_noalloc_slice(int64_t m, int64_t n) {
    const DirectShape d = direct_shape(m, n);
    constexpr int64_t cap = STK_DIRECT_NOALLOC_SCRATCH_BYTES / sizeof(double);
    const int64_t per_target = 3 * int64_t(d.nch);
    const int64_t ms = cap / per_target / 64 * 64;
    return ms < m ? ms : m;
}

void direct_sum_noalloc(const double *tgt, int64_t m, const double *src, int64_t n, const double *f,
                        const double *h, const double *nu, int32_t K, double *u_out, hipStream_t s) {
    const DirectShape d = direct_shape(m, n);
    const int64_t ms = direct_noalloc_slice(m, n);
    require(ms >= 1, "stk_direct_noalloc: n = " + std::to_string(n) + " sources need " +
                         std::to_string(3 * 64 * int64_t(d.nch) * int64_t(sizeof(double))) +
                         " bytes of partial sums per 64 targets, more than the fixed " +
                         std::to_string(STK_DIRECT_NOALLOC_SCRATCH_BYTES) + "-byte scratch array");
    int dev = -1;
    STK_HIP(hipGetDevice(&dev));
    double *part = scratch_on(dev);
    for (int r = 0; r < K; ++r)
        for (int64_t t0 = 0; t0 < m; t0 += ms) {
            const int64_t mm = m - t0 < ms ? m - t0 : ms;
            direct_launch(tgt + 3 * t0, mm, src, n, f + size_t(r) * n * 3, h + size_t(r) * n * 3, nu, d, part,
                          u_out + size_t(r) * m * 3 + 3 * t0, s);
        }
}

}  // namespace stk
