// ff_elementwise.hip -- elementwise float-float operators over SoA planes
// (Add22, Sub22, Mul22 with FMA or Dekker TwoProd, Div22) and the copy
// probe used as the bandwidth reference.
//
// Layout: four input planes and two output planes of n binary32 words.
// Each operator reads 16 bytes and writes 8 bytes per element and performs
// at most ~45 VALU operations, far below the gfx950 ridge point (~236
// binary32 operations per 24 bytes at 8 TB/s), so the kernels are
// HBM-bound.  One workgroup of kBlock (128) threads per block of kBlock *
// kPer (256) consecutive elements, in launch order; thread t takes elements
// b0 + t + kBlock k (k < kPer) of every plane, so each wavefront access is
// 256 contiguous bytes of a plane, issues all its non-temporal 4-byte loads
// before any arithmetic, and stores non-temporally.  Any 4-byte alignment.
// Below 2^22 elements (cache-resident) one float4 group per plane and thread
// instead, when the planes are 16-byte aligned.
#include "ff_device.h"
#include "ff_host.h"

namespace ffk {

// Operator tags: kernels are templated on these so that profiles name the
// operator (e.g. ffk::ew_stream<ffk::Add22>).
struct Add22 { static constexpr int op = ffd::OP_ADD; };
struct Sub22 { static constexpr int op = ffd::OP_SUB; };
struct Mul22 { static constexpr int op = ffd::OP_MUL; };
struct Mul22Dekker { static constexpr int op = ffd::OP_MUL_DEKKER; };
struct Div22 { static constexpr int op = ffd::OP_DIV; };
struct Add22Accurate { static constexpr int op = ffd::OP_ADD_ACCURATE; };
struct Sub22Accurate { static constexpr int op = ffd::OP_SUB_ACCURATE; };
struct Mul22Accurate { static constexpr int op = ffd::OP_MUL_ACCURATE; };
struct Div22Accurate { static constexpr int op = ffd::OP_DIV_ACCURATE; };

// Launch shape chosen by sweeps on MI355X at N = 2^28 (Add22, Mul22,
// Div22), each over five fresh allocations of the planes: small workgroups
// of kBlock = 128 threads by kPer = 2 lane-contiguous 4-byte elements moved
// 6.5-6.6 TB/s (0.97-0.98 ms per operator) whatever the planes' relative
// placement, against 6.2-6.35 TB/s for the earlier 1024 by 2 (which needed
// the planes' starts skewed by a few KiB to approach 6.4) and 6.1-6.4 TB/s
// for 256 or 512 by 2; 64 threads, 1 or 3 elements per thread, and 8-byte
// (float2) accesses per lane were all slower.  Issuing the loads plane by
// plane measured 1-1.5 % faster than element by element.
constexpr int kBlock = 128;   // 2 wavefronts of 64 lanes
constexpr int kPer = 2;       // elements per thread per plane
constexpr int64_t kSpan = static_cast<int64_t>(kBlock) * kPer;
// The float4 path for cache-resident sizes keeps 1024-thread workgroups.
constexpr int kVecBlock = 1024;

template <typename T>
__device__ __forceinline__ T ld_nt(const T *p) { return __builtin_nontemporal_load(p); }
template <typename T>
__device__ __forceinline__ void st_nt(T v, T *p) { __builtin_nontemporal_store(v, p); }

// The kPer lane-contiguous elements b0 + kBlock * k of one plane; zero
// past n.
__device__ __forceinline__ void load_plane(const float *p, int64_t b0, int64_t n,
                                           float (&v)[kPer])
{
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int64_t i = b0 + static_cast<int64_t>(kBlock) * k;
        v[k] = i < n ? ld_nt(p + i) : 0.0f;
    }
}

// No pointer is __restrict__: an output plane may be the same array as an
// input plane (in place).  Each element is loaded before it is stored, by
// the same thread, so in-place results equal out-of-place ones.
template <class Tag>
__global__ __launch_bounds__(kBlock) void ew_stream(const float *ah, const float *al,
                                                      const float *bh, const float *bl,
                                                      float *rh, float *rl, int64_t n)
{
    const int64_t b0 = static_cast<int64_t>(blockIdx.x) * kSpan + threadIdx.x;
    float xah[kPer], xal[kPer], xbh[kPer], xbl[kPer];
    // All loads are issued before any arithmetic, one plane at a time
    // (a.hi, b.hi, a.lo, b.lo): plane by plane measured 1-1.5 % faster than
    // element by element at N = 2^28.
    load_plane(ah, b0, n, xah);
    load_plane(bh, b0, n, xbh);
    load_plane(al, b0, n, xal);
    load_plane(bl, b0, n, xbl);
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int64_t i = b0 + static_cast<int64_t>(kBlock) * k;
        if (i < n) {
            float h, l;
            ffd::apply<Tag::op>(xah[k], xal[k], xbh[k], xbl[k], h, l);
            st_nt(h, rh + i);
            st_nt(l, rl + i);
        }
    }
}

// Below kSmallN elements the data sit in the 256 MB Infinity Cache and the
// launches are latency-bound; there one float4 group of every plane per
// thread (four times fewer load instructions) is as fast or faster (Add22 at
// 2^21: 7.6 against 8.6 us), while the lane-contiguous form wins from 2^22
// on (16.5 against 17.2 us).  The tail of n that is not a whole float4
// group runs in the lane-contiguous kernel.
constexpr int64_t kSmallN = int64_t(1) << 22;
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <class Tag>
__global__ __launch_bounds__(kVecBlock) void ew_vec(const f32x4 *ah, const f32x4 *al,
                                                   const f32x4 *bh, const f32x4 *bl, f32x4 *rh,
                                                   f32x4 *rl, int64_t nvec)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kVecBlock + threadIdx.x;
    if (i >= nvec)
        return;
    const f32x4 xah = ld_nt(ah + i), xal = ld_nt(al + i), xbh = ld_nt(bh + i),
                xbl = ld_nt(bl + i);
    f32x4 oh, ol;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        float h, l;
        ffd::apply<Tag::op>(xah[k], xal[k], xbh[k], xbl[k], h, l);
        oh[k] = h;
        ol[k] = l;
    }
    st_nt(oh, rh + i);
    st_nt(ol, rl + i);
}

// The copy probe (bandwidth reference and counter calibration): one plane
// in, one out, 512 threads by 4 lane-contiguous elements with non-temporal
// 4-byte loads (all issued first) and stores -- the fastest copy measured on
// MI355X at 2^28 words (6.41-6.45 TB/s, against 6.27 for one float4 group
// per lane and 5.7 for 1024 threads by 2).  Any 4-byte alignment.
constexpr int kCopyThreads = 512;
constexpr int kCopyPer = 4;

__global__ __launch_bounds__(kCopyThreads) void copy_stream(const float *src, float *dst,
                                                           int64_t n)
{
    const int64_t b0 =
        static_cast<int64_t>(blockIdx.x) * (kCopyThreads * kCopyPer) + threadIdx.x;
    float v[kCopyPer];
#pragma unroll
    for (int k = 0; k < kCopyPer; ++k) {
        const int64_t i = b0 + static_cast<int64_t>(kCopyThreads) * k;
        v[k] = i < n ? ld_nt(src + i) : 0.0f;
    }
#pragma unroll
    for (int k = 0; k < kCopyPer; ++k) {
        const int64_t i = b0 + static_cast<int64_t>(kCopyThreads) * k;
        if (i < n)
            st_nt(v[k], dst + i);
    }
}

template <class Tag>
ff_status elementwise(const float *ah, const float *al, const float *bh, const float *bl,
                      float *rh, float *rl, int64_t n, void *stream_ptr)
{
    if (n < 0)
        return FF_ERR_SIZE;
    if (n == 0)
        return FF_OK;
    if (!ah || !al || !bh || !bl || !rh || !rl)
        return FF_ERR_NULL;
    const void *ptrs[6] = {ah, al, bh, bl, rh, rl};
    for (const void *p : ptrs)
        if (!ffh::aligned(p, 4))
            return FF_ERR_ALIGN;
    hipStream_t stream = ffh::as_stream(stream_ptr);
    bool vec = n < kSmallN;
    for (const void *p : ptrs)
        vec = vec && ffh::aligned(p, 16);
    int64_t done = 0;
    if (vec) {
        const int64_t nvec = n / 4;
        done = 4 * nvec;
        if (nvec > 0)
            hipLaunchKernelGGL(ew_vec<Tag>, dim3(static_cast<unsigned>(ffh::cdiv(nvec, kVecBlock))),
                               dim3(kVecBlock), 0, stream, reinterpret_cast<const f32x4 *>(ah),
                               reinterpret_cast<const f32x4 *>(al),
                               reinterpret_cast<const f32x4 *>(bh),
                               reinterpret_cast<const f32x4 *>(bl), reinterpret_cast<f32x4 *>(rh),
                               reinterpret_cast<f32x4 *>(rl), nvec);
    }
    if (done < n) {
        const int64_t blocks = ffh::cdiv(n - done, kSpan);
        if (blocks > INT32_MAX)
            return FF_ERR_SIZE;
        hipLaunchKernelGGL(ew_stream<Tag>, dim3(static_cast<unsigned>(blocks)), dim3(kBlock), 0,
                           stream, ah + done, al + done, bh + done, bl + done, rh + done,
                           rl + done, n - done);
    }
    return ffh::launch_status();
}

} // namespace ffk

using namespace ffk;

extern "C" {

ff_status ff_add(const float *a_hi, const float *a_lo, const float *b_hi, const float *b_lo,
                 float *r_hi, float *r_lo, int64_t n, void *stream)
{
    return elementwise<Add22>(a_hi, a_lo, b_hi, b_lo, r_hi, r_lo, n, stream);
}

ff_status ff_sub(const float *a_hi, const float *a_lo, const float *b_hi, const float *b_lo,
                 float *r_hi, float *r_lo, int64_t n, void *stream)
{
    return elementwise<Sub22>(a_hi, a_lo, b_hi, b_lo, r_hi, r_lo, n, stream);
}

ff_status ff_mul(const float *a_hi, const float *a_lo, const float *b_hi, const float *b_lo,
                 float *r_hi, float *r_lo, int64_t n, void *stream)
{
    return elementwise<Mul22>(a_hi, a_lo, b_hi, b_lo, r_hi, r_lo, n, stream);
}

ff_status ff_mul_dekker(const float *a_hi, const float *a_lo, const float *b_hi,
                        const float *b_lo, float *r_hi, float *r_lo, int64_t n, void *stream)
{
    return elementwise<Mul22Dekker>(a_hi, a_lo, b_hi, b_lo, r_hi, r_lo, n, stream);
}

ff_status ff_div(const float *a_hi, const float *a_lo, const float *b_hi, const float *b_lo,
                 float *r_hi, float *r_lo, int64_t n, void *stream)
{
    return elementwise<Div22>(a_hi, a_lo, b_hi, b_lo, r_hi, r_lo, n, stream);
}

ff_status ff_add_accurate(const float *a_hi, const float *a_lo, const float *b_hi,
                          const float *b_lo, float *r_hi, float *r_lo, int64_t n, void *stream)
{
    return elementwise<Add22Accurate>(a_hi, a_lo, b_hi, b_lo, r_hi, r_lo, n, stream);
}

ff_status ff_sub_accurate(const float *a_hi, const float *a_lo, const float *b_hi,
                          const float *b_lo, float *r_hi, float *r_lo, int64_t n, void *stream)
{
    return elementwise<Sub22Accurate>(a_hi, a_lo, b_hi, b_lo, r_hi, r_lo, n, stream);
}

ff_status ff_mul_accurate(const float *a_hi, const float *a_lo, const float *b_hi,
                          const float *b_lo, float *r_hi, float *r_lo, int64_t n, void *stream)
{
    return elementwise<Mul22Accurate>(a_hi, a_lo, b_hi, b_lo, r_hi, r_lo, n, stream);
}

ff_status ff_div_accurate(const float *a_hi, const float *a_lo, const float *b_hi,
                          const float *b_lo, float *r_hi, float *r_lo, int64_t n, void *stream)
{
    return elementwise<Div22Accurate>(a_hi, a_lo, b_hi, b_lo, r_hi, r_lo, n, stream);
}

ff_status ff_copy(const float *src, float *dst, int64_t n, void *stream_ptr)
{
    if (n < 0)
        return FF_ERR_SIZE;
    if (n == 0)
        return FF_OK;
    if (!src || !dst)
        return FF_ERR_NULL;
    if (!ffh::aligned(src, 4) || !ffh::aligned(dst, 4))
        return FF_ERR_ALIGN;
    const int64_t blocks = ffh::cdiv(n, int64_t(kCopyThreads) * kCopyPer);
    if (blocks > INT32_MAX)
        return FF_ERR_SIZE;
    hipLaunchKernelGGL(copy_stream, dim3(static_cast<unsigned>(blocks)), dim3(kCopyThreads), 0,
                       ffh::as_stream(stream_ptr), src, dst, n);
    return ffh::launch_status();
}

} // extern "C"
