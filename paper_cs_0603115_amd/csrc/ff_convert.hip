// ff_convert.hip -- conversions between binary64 and float-float planes.
//
// The paper's operators take float-float inputs; these move data in and
// out of that format on the device:
//   from binary64: hi = fl32(x), lo = fl32(x - hi).  hi is x rounded to 24
//     bits, so x - hi is exact in binary64 and hi + lo is x to within
//     2^-48 |x| (|x| below the binary32 overflow threshold, normal range).
//   to binary64:   x = (double) hi + (double) lo, one binary64 rounding,
//     exact whenever the pair's bits fit in 53.
// 16 bytes per element either way; HBM-bound.  Lane-contiguous accesses
// (each wavefront load or store is one contiguous segment of a plane), all
// loads of a thread issued before the arithmetic, non-temporal loads and
// stores; any 4-byte (binary32) and 8-byte (binary64) alignment.  Shapes from
// sweeps on MI355X at N = 2^28: from binary64, 128 threads by 2 elements
// (6.6 TB/s, against 6.3 for 256 by 4 and 5.9 for one float4 group per plane
// and lane); to binary64, 1024 threads by one element (6.0 TB/s; 128- and
// 256-thread workgroups by 2 or 4 elements reached 4.8-5.1).
#include "ff_device.h"
#include "ff_host.h"

namespace ffk {

constexpr int kFromThreads = 128, kFromPer = 2;
constexpr int kToThreads = 1024, kToPer = 1;

__device__ __forceinline__ void split_f64(double x, float &hi, float &lo)
{
    hi = static_cast<float>(x);
    lo = static_cast<float>(x - static_cast<double>(hi));
}

__device__ __forceinline__ double join_f64(float hi, float lo)
{
    return static_cast<double>(hi) + static_cast<double>(lo);
}

__global__ __launch_bounds__(kFromThreads) void from_f64_kernel(const double *__restrict__ x,
                                                                float *__restrict__ hi,
                                                                float *__restrict__ lo, int64_t n)
{
    const int64_t b0 =
        static_cast<int64_t>(blockIdx.x) * (kFromThreads * kFromPer) + threadIdx.x;
    double v[kFromPer];
#pragma unroll
    for (int k = 0; k < kFromPer; ++k) {
        const int64_t i = b0 + static_cast<int64_t>(kFromThreads) * k;
        v[k] = i < n ? __builtin_nontemporal_load(x + i) : 0.0;
    }
#pragma unroll
    for (int k = 0; k < kFromPer; ++k) {
        const int64_t i = b0 + static_cast<int64_t>(kFromThreads) * k;
        if (i < n) {
            float h, l;
            split_f64(v[k], h, l);
            __builtin_nontemporal_store(h, hi + i);
            __builtin_nontemporal_store(l, lo + i);
        }
    }
}

__global__ __launch_bounds__(kToThreads) void to_f64_kernel(const float *__restrict__ hi,
                                                            const float *__restrict__ lo,
                                                            double *__restrict__ x, int64_t n)
{
    const int64_t b0 = static_cast<int64_t>(blockIdx.x) * (kToThreads * kToPer) + threadIdx.x;
    float h[kToPer], l[kToPer];
#pragma unroll
    for (int k = 0; k < kToPer; ++k) {
        const int64_t i = b0 + static_cast<int64_t>(kToThreads) * k;
        h[k] = i < n ? __builtin_nontemporal_load(hi + i) : 0.0f;
    }
#pragma unroll
    for (int k = 0; k < kToPer; ++k) {
        const int64_t i = b0 + static_cast<int64_t>(kToThreads) * k;
        l[k] = i < n ? __builtin_nontemporal_load(lo + i) : 0.0f;
    }
#pragma unroll
    for (int k = 0; k < kToPer; ++k) {
        const int64_t i = b0 + static_cast<int64_t>(kToThreads) * k;
        if (i < n)
            __builtin_nontemporal_store(join_f64(h[k], l[k]), x + i);
    }
}

// Shared argument checks: sizes, null pointers, 4-byte (binary32) and
// 8-byte (binary64) alignment.
static ff_status check_planes(const void *f64, const void *hi, const void *lo, int64_t n)
{
    if (n < 0)
        return FF_ERR_SIZE;
    if (n == 0)
        return FF_OK;
    if (!f64 || !hi || !lo)
        return FF_ERR_NULL;
    if (!ffh::aligned(f64, 8) || !ffh::aligned(hi, 4) || !ffh::aligned(lo, 4))
        return FF_ERR_ALIGN;
    return FF_OK;
}

} // namespace ffk

using namespace ffk;

extern "C" {

ff_status ff_from_f64(const double *x, float *hi, float *lo, int64_t n, void *stream)
{
    const ff_status st = check_planes(x, hi, lo, n);
    if (st != FF_OK || n == 0)
        return st;
    const int64_t blocks = ffh::cdiv(n, int64_t(kFromThreads) * kFromPer);
    if (blocks > INT32_MAX)
        return FF_ERR_SIZE;
    hipLaunchKernelGGL(from_f64_kernel, dim3(static_cast<unsigned>(blocks)), dim3(kFromThreads), 0,
                       ffh::as_stream(stream), x, hi, lo, n);
    return ffh::launch_status();
}

ff_status ff_to_f64(const float *hi, const float *lo, double *x, int64_t n, void *stream)
{
    const ff_status st = check_planes(x, hi, lo, n);
    if (st != FF_OK || n == 0)
        return st;
    const int64_t blocks = ffh::cdiv(n, int64_t(kToThreads) * kToPer);
    if (blocks > INT32_MAX)
        return FF_ERR_SIZE;
    hipLaunchKernelGGL(to_f64_kernel, dim3(static_cast<unsigned>(blocks)), dim3(kToThreads), 0,
                       ffh::as_stream(stream), hi, lo, x, n);
    return ffh::launch_status();
}

} // extern "C"
