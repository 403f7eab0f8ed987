// ff_paper_ops.hip -- the error-free transforms and binary32 reference
// operators that the paper times beside its float-float operators (section
// 6, Tables 3 and 4), as stream kernels over SoA planes:
//   Add12 (section 4.1, Add12 theorem; the six-operation form),
//   Mul12 with FMA TwoProd or with Dekker's Split (Mul12 theorem),
//   binary32 add, multiply and multiply-add (one rounding).
//
// Same streaming structure as the float-float operators: workgroups in
// launch order, lane-contiguous elements (128 threads by 2 per plane, or 256
// by 4 for binary32 Add and Mul), all 4-byte
// non-temporal loads issued before the arithmetic (plane by plane where the
// kernel writes two planes), any 4-byte alignment; one float4 group per plane
// and thread below 2^22 elements.  Bytes per element: 12 (add, mul), 16 (mad,
// Add12, Mul12); all HBM-bound at large n, launch-bound at the paper's sizes.
#include "ff_device.h"
#include "ff_host.h"

namespace ffk {

constexpr int kStreamBlock = 1024;   // workgroup of the float4 form (below 2^22)

// An operator maps IN binary32 inputs of one element to OUT outputs.
struct OpAdd12 {
    static constexpr int kIn = 2, kOut = 2;
    __device__ __forceinline__ static void apply(const float *x, float *y)
    {
        ffd::add12(x[0], x[1], y[0], y[1]);
    }
};
struct OpMul12Fma {
    static constexpr int kIn = 2, kOut = 2;
    __device__ __forceinline__ static void apply(const float *x, float *y)
    {
        ffd::mul12_fma(x[0], x[1], y[0], y[1]);
    }
};
struct OpMul12Dekker {
    static constexpr int kIn = 2, kOut = 2;
    __device__ __forceinline__ static void apply(const float *x, float *y)
    {
        ffd::mul12_dekker(x[0], x[1], y[0], y[1]);
    }
};
struct OpF32Add {
    static constexpr int kIn = 2, kOut = 1;
    __device__ __forceinline__ static void apply(const float *x, float *y) { y[0] = x[0] + x[1]; }
};
struct OpF32Mul {
    static constexpr int kIn = 2, kOut = 1;
    __device__ __forceinline__ static void apply(const float *x, float *y) { y[0] = x[0] * x[1]; }
};
struct OpF32Mad {
    static constexpr int kIn = 3, kOut = 1;
    __device__ __forceinline__ static void apply(const float *x, float *y)
    {
        y[0] = __builtin_fmaf(x[0], x[1], x[2]);
    }
};

template <int IN, int OUT>
struct StreamPlanes {
    const float *in[IN];
    float *out[OUT];
};

typedef float f32x4 __attribute__((ext_vector_type(4)));

// Below kStreamSmallN elements (cache-resident, latency-bound launches) one
// float4 group of every plane per thread is faster, as for the float-float
// operators; the tail that is not a whole group and larger n run the
// lane-contiguous kernel.
constexpr int64_t kStreamSmallN = int64_t(1) << 22;

template <class Op>
__global__ __launch_bounds__(kStreamBlock) void stream_vec(StreamPlanes<Op::kIn, Op::kOut> p,
                                                           int64_t nvec)
{
    const int64_t g = static_cast<int64_t>(blockIdx.x) * kStreamBlock + threadIdx.x;
    if (g >= nvec)
        return;
    f32x4 x[Op::kIn], y[Op::kOut];
#pragma unroll
    for (int k = 0; k < Op::kIn; ++k)
        x[k] = __builtin_nontemporal_load(reinterpret_cast<const f32x4 *>(p.in[k]) + g);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        float xi[Op::kIn], yo[Op::kOut];
#pragma unroll
        for (int k = 0; k < Op::kIn; ++k)
            xi[k] = x[k][c];
        Op::apply(xi, yo);
#pragma unroll
        for (int k = 0; k < Op::kOut; ++k)
            y[k][c] = yo[k];
    }
#pragma unroll
    for (int k = 0; k < Op::kOut; ++k)
        __builtin_nontemporal_store(y[k], reinterpret_cast<f32x4 *>(p.out[k]) + g);
}

// Launch shape of the lane-contiguous form, from sweeps at N = 2^28: the
// float-float operators' 128 threads by 2 elements for Add12 and Mul12 (two
// output planes; 6.4 TB/s, against 6.2 for 1024 by 2) and for the
// three-input Mad (6.6 TB/s, against 6.3 for 256 by 4); 256 by 4 for the
// two-input, one-output binary32 Add and Mul (6.4 TB/s; 128 by 4 ties, 128
// by 2 is 2 % slower).
template <class Op>
struct StreamShape {
    static constexpr bool kWide = Op::kOut == 1 && Op::kIn == 2;
    static constexpr int kBlock = kWide ? 256 : 128;
    static constexpr int kPer = kWide ? 4 : 2;   // elements per thread per plane
    static constexpr int64_t kSpan = static_cast<int64_t>(kBlock) * kPer;
};

template <class Op>
__global__ __launch_bounds__(StreamShape<Op>::kBlock) void stream_op_kernel(
    StreamPlanes<Op::kIn, Op::kOut> p, int64_t n)
{
    using Sh = StreamShape<Op>;
    const int64_t b0 = static_cast<int64_t>(blockIdx.x) * Sh::kSpan + threadIdx.x;
    float x[Sh::kPer][Op::kIn];
    // Every load is issued before any arithmetic.  Measured at N = 2^26 and
    // 2^28: with two output planes, issuing the loads one input plane at a
    // time is 1 % faster than element by element; with one output plane it
    // is 3-5 % slower, so those kernels keep the element order.
    if constexpr (Op::kOut >= 2) {
#pragma unroll
        for (int q = 0; q < Op::kIn; ++q) {
#pragma unroll
            for (int k = 0; k < Sh::kPer; ++k) {
                const int64_t i = b0 + static_cast<int64_t>(Sh::kBlock) * k;
                x[k][q] = i < n ? __builtin_nontemporal_load(p.in[q] + i) : 0.0f;
            }
        }
    } else {
#pragma unroll
        for (int k = 0; k < Sh::kPer; ++k) {
            const int64_t i = b0 + static_cast<int64_t>(Sh::kBlock) * k;
#pragma unroll
            for (int q = 0; q < Op::kIn; ++q)
                x[k][q] = i < n ? __builtin_nontemporal_load(p.in[q] + i) : 0.0f;
        }
    }
#pragma unroll
    for (int k = 0; k < Sh::kPer; ++k) {
        const int64_t i = b0 + static_cast<int64_t>(Sh::kBlock) * k;
        if (i < n) {
            float y[Op::kOut];
            Op::apply(x[k], y);
#pragma unroll
            for (int q = 0; q < Op::kOut; ++q)
                __builtin_nontemporal_store(y[q], p.out[q] + i);
        }
    }
}

template <class Op>
ff_status stream_op(StreamPlanes<Op::kIn, Op::kOut> p, int64_t n, void *stream_ptr)
{
    if (n < 0)
        return FF_ERR_SIZE;
    if (n == 0)
        return FF_OK;
    for (int k = 0; k < Op::kIn; ++k) {
        if (!p.in[k])
            return FF_ERR_NULL;
        if (!ffh::aligned(p.in[k], 4))
            return FF_ERR_ALIGN;
    }
    for (int k = 0; k < Op::kOut; ++k) {
        if (!p.out[k])
            return FF_ERR_NULL;
        if (!ffh::aligned(p.out[k], 4))
            return FF_ERR_ALIGN;
    }
    hipStream_t st = ffh::as_stream(stream_ptr);
    bool vec = n < kStreamSmallN;
    for (int k = 0; k < Op::kIn; ++k)
        vec = vec && ffh::aligned(p.in[k], 16);
    for (int k = 0; k < Op::kOut; ++k)
        vec = vec && ffh::aligned(p.out[k], 16);
    int64_t done = 0;
    if (vec) {
        const int64_t nvec = n / 4;
        done = 4 * nvec;
        if (nvec > 0)
            hipLaunchKernelGGL(stream_vec<Op>,
                               dim3(static_cast<unsigned>(ffh::cdiv(nvec, kStreamBlock))),
                               dim3(kStreamBlock), 0, st, p, nvec);
    }
    if (done < n) {
        StreamPlanes<Op::kIn, Op::kOut> rest = p;
        for (int k = 0; k < Op::kIn; ++k)
            rest.in[k] += done;
        for (int k = 0; k < Op::kOut; ++k)
            rest.out[k] += done;
        const int64_t blocks = ffh::cdiv(n - done, StreamShape<Op>::kSpan);
        if (blocks > INT32_MAX)
            return FF_ERR_SIZE;
        hipLaunchKernelGGL(stream_op_kernel<Op>, dim3(static_cast<unsigned>(blocks)),
                           dim3(StreamShape<Op>::kBlock), 0, st, rest, n - done);
    }
    return ffh::launch_status();
}

} // namespace ffk

using namespace ffk;

extern "C" {

ff_status ff_add12(const float *a, const float *b, float *s, float *r, int64_t n, void *stream)
{
    return stream_op<OpAdd12>(StreamPlanes<2, 2>{{a, b}, {s, r}}, n, stream);
}

ff_status ff_mul12(const float *a, const float *b, float *x, float *y, int64_t n, void *stream)
{
    return stream_op<OpMul12Fma>(StreamPlanes<2, 2>{{a, b}, {x, y}}, n, stream);
}

ff_status ff_mul12_dekker(const float *a, const float *b, float *x, float *y, int64_t n,
                          void *stream)
{
    return stream_op<OpMul12Dekker>(StreamPlanes<2, 2>{{a, b}, {x, y}}, n, stream);
}

ff_status ff_f32_add(const float *a, const float *b, float *r, int64_t n, void *stream)
{
    return stream_op<OpF32Add>(StreamPlanes<2, 1>{{a, b}, {r}}, n, stream);
}

ff_status ff_f32_mul(const float *a, const float *b, float *r, int64_t n, void *stream)
{
    return stream_op<OpF32Mul>(StreamPlanes<2, 1>{{a, b}, {r}}, n, stream);
}

ff_status ff_f32_mad(const float *a, const float *b, const float *c, float *r, int64_t n,
                     void *stream)
{
    return stream_op<OpF32Mad>(StreamPlanes<3, 1>{{a, b, c}, {r}}, n, stream);
}

} // extern "C"
