// The per-step history sum on caller buffers with no device allocation: the
// partial sums of the lag splits live in a fixed device array of the library
// instead of a buffer allocated per call (include/qhp.h,
// qhp_history_sum_noalloc).
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/qhp.h"
#include "march.h"

namespace {

constexpr size_t kScratchBytes = (size_t)QHP_NOALLOC_SCRATCH_MB << 20;

// Partial sums of the no-allocation history sum.  Every GPU the library runs
// on holds its own copy until the process ends.  Host code never passes this
// name to a kernel or a copy: it stands for the host-side shadow, not the
// device address.  The address on each device comes from hipGetSymbolAddress.
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

constexpr int kMaxDevices = 64;
std::mutex g_mutex;
void *g_scratch[kMaxDevices] = {};  // device address of `scratch` on each device, once looked up

// the array's address on `dev`, looked up once with that device current
hipError_t scratch_on(int dev, void **out)
{
    std::lock_guard<std::mutex> lock(g_mutex);
    if (!g_scratch[dev]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != dev && (e = hipSetDevice(dev)) != hipSuccess) return e;
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != dev) (void)hipSetDevice(cur);
        if (e != hipSuccess) return e;
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return hipSuccess;
}

}  // namespace

extern "C" int qhp_history_sum_noalloc(void *stream, int32_t precision, int64_t ne, int64_t ld, int64_t nrhs,
                                       int64_t kmax, const void *slabs, const float *scales, const void *ring,
                                       int64_t n_slots, int64_t head, const double *r, double *b, int32_t variant)
{
    if (!qhp::history_args_valid(precision, ne, ld, nrhs, kmax, slabs, scales, ring, n_slots, head, r, b, variant))
        return QHP_EINVAL;
    const int nsplit = qhp::history_split_count(precision, ne, nrhs, kmax, variant);
    if ((size_t)nsplit * (size_t)ne * (size_t)nrhs * sizeof(double) > kScratchBytes) return QHP_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    int dev = -1;
    if (s) {
        if (hipStreamGetDevice(s, &dev) != hipSuccess) return QHP_EDEVICE;
    } else if (hipGetDevice(&dev) != hipSuccess) {
        return QHP_EDEVICE;
    }
    if (dev < 0 || dev >= kMaxDevices) return QHP_EDEVICE;
    void *partial = nullptr;
    if (scratch_on(dev, &partial) != hipSuccess || !partial) {
        (void)hipGetLastError();
        return QHP_EDEVICE;
    }
    qhp::launch_history(s, precision, ne, ld, nrhs, kmax, slabs, precision == QHP_BF16 ? scales : nullptr, ring,
                        n_slots, head, r, b, partial, nsplit, nullptr, nullptr, variant);
    return hipGetLastError() == hipSuccess ? QHP_OK : QHP_EDEVICE;
}
