// The allocation-free FP64 inner product (el_dot_f64_noalloc).
//
// el_dot_f64 keeps its partial sums in the plan's workspace, which the caller
// allocated.  Callers that can neither allocate device memory nor hold a plan
// (code under stream capture, tight serving loops) use this variant: the same
// two kernels (k_dot_partial, k_dot_final) with the partial sums in `scratch`,
// a static device array of the library.  Each GPU the library runs on holds its
// own copy of the array until the process ends; its device address is looked
// up once per device and kept.
#include <mutex>
#include <vector>

#include "el_impl.h"

// Partial sums of the dot kernels: one double per block (8 KiB), every one written by each
// call before it is read, so nothing needs clearing between calls.  In host code the name
// stands for a host-side shadow: kernels receive the address scratch_of() looked up.
static __device__ __align__(256) double scratch[el::kDotBlocks];

namespace {

// Largest element count accepted (the reduction itself has no size limit: the grid-stride
// loop of k_dot_partial folds any n into the kDotBlocks partial sums).
constexpr long long kDotNoallocMax = 1LL << 40;

std::mutex g_mu;
std::vector<double *> g_ptr;   // device address of scratch per device (null: not looked up yet)

// Device address of this device's scratch (the device is current).
el_status scratch_of(int dev, double **out) {
    std::lock_guard<std::mutex> lock(g_mu);
    if (g_ptr.empty()) {
        int n = 0;
        const hipError_t e = hipGetDeviceCount(&n);
        if (e != hipSuccess) return el::set_error(EL_EDEVICE, "hipGetDeviceCount: %s", hipGetErrorString(e));
        g_ptr.assign(n > 0 ? n : 1, nullptr);
    }
    if (dev < 0 || dev >= (int)g_ptr.size()) return el::set_error(EL_EDEVICE, "device %d outside the device count", dev);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return el::set_error(EL_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_ptr[dev] = static_cast<double *>(p);
    }
    *out = g_ptr[dev];
    return EL_OK;
}

}  // namespace

extern "C" {

el_status el_dot_f64_noalloc(int32_t precision, int64_t n, const void *a, const void *b, double *out, void *stream) {
    if (precision != EL_F32 && precision != EL_F64) return el::set_error(EL_EINVAL, "precision must be EL_F32 or EL_F64");
    if (n < 0 || n > kDotNoallocMax)
        return el::set_error(EL_EINVAL, "n = %lld outside 0..%lld", (long long)n, (long long)kDotNoallocMax);
    if (!out || (n > 0 && (!a || !b))) return el::set_error(EL_EINVAL, "a, b or out is NULL");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return el::set_error(EL_EDEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    double *partial = nullptr;
    const el_status st = scratch_of(dev, &partial);
    if (st != EL_OK) return st;
    const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    e = precision == EL_F64
            ? el::launch_dot(static_cast<const double *>(a), static_cast<const double *>(b), (long long)n, partial, out, s)
            : el::launch_dot(static_cast<const float *>(a), static_cast<const float *>(b), (long long)n, partial, out, s);
    if (e != hipSuccess) return el::set_error(EL_EDEVICE, "dot: %s", hipGetErrorString(e));
    return EL_OK;
}

}  // extern "C"
