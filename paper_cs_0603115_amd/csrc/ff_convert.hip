// ff_convert.hip -- conversions between binary64 and float-float planes.
//
// The paper's operators take float-float inputs; these move data in and
// out of that format on the device:
//   from binary64: hi = fl32(x), lo = fl32(x - hi).  hi is x rounded to 24
//     bits, so x - hi is exact in binary64 and hi + lo is x to within
//     2^-48 |x| (|x| below the binary32 overflow threshold, normal range).
//   to binary64:   x = (double) hi + (double) lo, one binary64 rounding,
//     exact whenever the pair's bits fit in 53.
// 16 bytes per element either way; HBM-bound.  Four elements per lane when
// every plane is 16-byte aligned (two 16-byte loads or stores of binary64,
// one of each binary32 plane), one per lane otherwise and for the tail.
#include "ff_device.h"
#include "ff_host.h"

namespace ffk {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

constexpr int kConvBlock = 256;

__device__ __forceinline__ void split_f64(double x, float &hi, float &lo)
{
    hi = static_cast<float>(x);
    lo = static_cast<float>(x - static_cast<double>(hi));
}

__device__ __forceinline__ double join_f64(float hi, float lo)
{
    return static_cast<double>(hi) + static_cast<double>(lo);
}

__global__ __launch_bounds__(kConvBlock) void from_f64_vec(const f64x2 *__restrict__ x,
                                                           f32x4 *__restrict__ hi,
                                                           f32x4 *__restrict__ lo, int64_t ngroups)
{
    const int64_t g = static_cast<int64_t>(blockIdx.x) * kConvBlock + threadIdx.x;
    if (g >= ngroups)
        return;
    const f64x2 a = __builtin_nontemporal_load(x + 2 * g);
    const f64x2 b = __builtin_nontemporal_load(x + 2 * g + 1);
    const double v[4] = {a[0], a[1], b[0], b[1]};
    f32x4 h, l;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        float hc, lc;
        split_f64(v[c], hc, lc);
        h[c] = hc;
        l[c] = lc;
    }
    __builtin_nontemporal_store(h, hi + g);
    __builtin_nontemporal_store(l, lo + g);
}

__global__ __launch_bounds__(kConvBlock) void from_f64_scalar(const double *__restrict__ x,
                                                              float *__restrict__ hi,
                                                              float *__restrict__ lo, int64_t n)
{
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kConvBlock;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kConvBlock + threadIdx.x; i < n;
         i += stride)
        split_f64(x[i], hi[i], lo[i]);
}

__global__ __launch_bounds__(kConvBlock) void to_f64_vec(const f32x4 *__restrict__ hi,
                                                         const f32x4 *__restrict__ lo,
                                                         f64x2 *__restrict__ x, int64_t ngroups)
{
    const int64_t g = static_cast<int64_t>(blockIdx.x) * kConvBlock + threadIdx.x;
    if (g >= ngroups)
        return;
    const f32x4 h = __builtin_nontemporal_load(hi + g);
    const f32x4 l = __builtin_nontemporal_load(lo + g);
    const f64x2 a = {join_f64(h[0], l[0]), join_f64(h[1], l[1])};
    const f64x2 b = {join_f64(h[2], l[2]), join_f64(h[3], l[3])};
    __builtin_nontemporal_store(a, x + 2 * g);
    __builtin_nontemporal_store(b, x + 2 * g + 1);
}

__global__ __launch_bounds__(kConvBlock) void to_f64_scalar(const float *__restrict__ hi,
                                                            const float *__restrict__ lo,
                                                            double *__restrict__ x, int64_t n)
{
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kConvBlock;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kConvBlock + threadIdx.x; i < n;
         i += stride)
        x[i] = join_f64(hi[i], lo[i]);
}

// Shared argument checks: sizes, null pointers, 4-byte (binary32) and
// 8-byte (binary64) alignment; returns whether the float4 path applies.
static ff_status check_planes(const void *f64, const void *hi, const void *lo, int64_t n,
                              bool &vec)
{
    if (n < 0)
        return FF_ERR_SIZE;
    if (n == 0)
        return FF_OK;
    if (!f64 || !hi || !lo)
        return FF_ERR_NULL;
    if (!ffh::aligned(f64, 8) || !ffh::aligned(hi, 4) || !ffh::aligned(lo, 4))
        return FF_ERR_ALIGN;
    vec = ffh::aligned(f64, 16) && ffh::aligned(hi, 16) && ffh::aligned(lo, 16);
    return FF_OK;
}

static unsigned scalar_grid(int64_t n)
{
    const int64_t blocks = ffh::cdiv(n, kConvBlock);
    return static_cast<unsigned>(blocks < 65536 ? blocks : 65536);
}

} // namespace ffk

using namespace ffk;

extern "C" {

ff_status ff_from_f64(const double *x, float *hi, float *lo, int64_t n, void *stream)
{
    bool vec = false;
    const ff_status st = check_planes(x, hi, lo, n, vec);
    if (st != FF_OK || n == 0)
        return st;
    hipStream_t s = ffh::as_stream(stream);
    int64_t done = 0;
    if (vec) {
        const int64_t ngroups = n / 4;
        done = 4 * ngroups;
        if (ngroups > 0) {
            const int64_t blocks = ffh::cdiv(ngroups, kConvBlock);
            if (blocks > INT32_MAX)
                return FF_ERR_SIZE;
            hipLaunchKernelGGL(from_f64_vec, dim3(static_cast<unsigned>(blocks)), dim3(kConvBlock),
                               0, s, reinterpret_cast<const f64x2 *>(x),
                               reinterpret_cast<f32x4 *>(hi), reinterpret_cast<f32x4 *>(lo),
                               ngroups);
        }
    }
    if (done < n)
        hipLaunchKernelGGL(from_f64_scalar, dim3(scalar_grid(n - done)), dim3(kConvBlock), 0, s,
                           x + done, hi + done, lo + done, n - done);
    return ffh::launch_status();
}

ff_status ff_to_f64(const float *hi, const float *lo, double *x, int64_t n, void *stream)
{
    bool vec = false;
    const ff_status st = check_planes(x, hi, lo, n, vec);
    if (st != FF_OK || n == 0)
        return st;
    hipStream_t s = ffh::as_stream(stream);
    int64_t done = 0;
    if (vec) {
        const int64_t ngroups = n / 4;
        done = 4 * ngroups;
        if (ngroups > 0) {
            const int64_t blocks = ffh::cdiv(ngroups, kConvBlock);
            if (blocks > INT32_MAX)
                return FF_ERR_SIZE;
            hipLaunchKernelGGL(to_f64_vec, dim3(static_cast<unsigned>(blocks)), dim3(kConvBlock), 0,
                               s, reinterpret_cast<const f32x4 *>(hi),
                               reinterpret_cast<const f32x4 *>(lo), reinterpret_cast<f64x2 *>(x),
                               ngroups);
        }
    }
    if (done < n)
        hipLaunchKernelGGL(to_f64_scalar, dim3(scalar_grid(n - done)), dim3(kConvBlock), 0, s,
                           hi + done, lo + done, x + done, n - done);
    return ffh::launch_status();
}

} // extern "C"
