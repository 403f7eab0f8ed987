// ff_elementwise.hip -- elementwise float-float operators over SoA planes
// (Add22, Sub22, Mul22 with FMA or Dekker TwoProd, Div22) and the copy
// probe used as the bandwidth reference.
//
// Layout: four input planes and two output planes of n binary32 words.
// Each operator reads 16 bytes and writes 8 bytes per element and performs
// at most ~45 VALU operations, far below the gfx950 ridge point (~118 lane
// operations per 24 bytes at 8 TB/s), so the kernels are HBM-bound.  The
// fast path streams the planes with 16-byte non-temporal loads and stores:
// every thread owns kUnroll float4 groups of each plane, the groups of a
// workgroup are contiguous, and consecutive lanes touch consecutive 16-byte
// words so that each wavefront instruction moves 1 KiB per plane.
#include "ff_device.h"
#include "ff_host.h"

namespace ffk {

typedef float f32x4 __attribute__((ext_vector_type(4)));

// Operator tags: kernels are templated on these so that profiles name the
// operator (e.g. ffk::ew_vec<ffk::Add22>).
struct Add22 { static constexpr int op = ffd::OP_ADD; };
struct Sub22 { static constexpr int op = ffd::OP_SUB; };
struct Mul22 { static constexpr int op = ffd::OP_MUL; };
struct Mul22Dekker { static constexpr int op = ffd::OP_MUL_DEKKER; };
struct Div22 { static constexpr int op = ffd::OP_DIV; };
struct Add22Accurate { static constexpr int op = ffd::OP_ADD_ACCURATE; };
struct Sub22Accurate { static constexpr int op = ffd::OP_SUB_ACCURATE; };
struct Mul22Accurate { static constexpr int op = ffd::OP_MUL_ACCURATE; };
struct Div22Accurate { static constexpr int op = ffd::OP_DIV_ACCURATE; };

// Launch shape chosen by a sweep on MI355X over workgroup sizes 256-1024,
// 1-8 float4 groups per thread, persistent grids, XCD-contiguous tile
// orders and plane base offsets: 1024 threads with one float4 group per
// plane per thread reached 6.1 TB/s for every operator (the plain copy probe
// of the same pattern: 6.3 TB/s).
constexpr int kBlock = 1024;  // 16 wavefronts of 64 lanes
constexpr int kUnroll = 1;    // float4 groups per thread per plane

template <typename T>
__device__ __forceinline__ T ld_nt(const T *p) { return __builtin_nontemporal_load(p); }
template <typename T>
__device__ __forceinline__ void st_nt(T v, T *p) { __builtin_nontemporal_store(v, p); }

template <int OP>
__device__ __forceinline__ void apply4(const f32x4 &ah, const f32x4 &al, const f32x4 &bh,
                                       const f32x4 &bl, f32x4 &rh, f32x4 &rl)
{
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        float h, l;
        ffd::apply<OP>(ah[k], al[k], bh[k], bl[k], h, l);
        rh[k] = h;
        rl[k] = l;
    }
}

// Vector path: planes 16-byte aligned; element groups [0, nvec) of 4 floats.
// Workgroup w owns groups [w*kBlock*kUnroll, (w+1)*kBlock*kUnroll); lane t
// of the workgroup takes groups t, t + kBlock, ... so each load instruction
// of a wavefront is one contiguous 1 KiB segment.
template <class Tag>
__global__ __launch_bounds__(kBlock) void ew_vec(const f32x4 *__restrict__ ah,
                                                   const f32x4 *__restrict__ al,
                                                   const f32x4 *__restrict__ bh,
                                                   const f32x4 *__restrict__ bl,
                                                   f32x4 *__restrict__ rh,
                                                   f32x4 *__restrict__ rl, int64_t nvec)
{
    const int64_t first = static_cast<int64_t>(blockIdx.x) * (kBlock * kUnroll) + threadIdx.x;
    f32x4 xah[kUnroll], xal[kUnroll], xbh[kUnroll], xbl[kUnroll];
    if (static_cast<int64_t>(blockIdx.x + 1) * (kBlock * kUnroll) <= nvec) {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const int64_t i = first + u * kBlock;
            xah[u] = ld_nt(ah + i);
            xal[u] = ld_nt(al + i);
            xbh[u] = ld_nt(bh + i);
            xbl[u] = ld_nt(bl + i);
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const int64_t i = first + u * kBlock;
            f32x4 oh, ol;
            apply4<Tag::op>(xah[u], xal[u], xbh[u], xbl[u], oh, ol);
            st_nt(oh, rh + i);
            st_nt(ol, rl + i);
        }
    } else {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const int64_t i = first + u * kBlock;
            if (i < nvec) {
                f32x4 oh, ol;
                apply4<Tag::op>(ld_nt(ah + i), ld_nt(al + i), ld_nt(bh + i), ld_nt(bl + i), oh, ol);
                st_nt(oh, rh + i);
                st_nt(ol, rl + i);
            }
        }
    }
}

// Scalar path: any 4-byte alignment, grid-stride over [0, n).
template <class Tag>
__global__ __launch_bounds__(kBlock) void ew_scalar(const float *__restrict__ ah,
                                                      const float *__restrict__ al,
                                                      const float *__restrict__ bh,
                                                      const float *__restrict__ bl,
                                                      float *__restrict__ rh,
                                                      float *__restrict__ rl, int64_t n)
{
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n; i += stride) {
        float h, l;
        ffd::apply<Tag::op>(ah[i], al[i], bh[i], bl[i], h, l);
        rh[i] = h;
        rl[i] = l;
    }
}

__global__ __launch_bounds__(kBlock) void copy_vec(const f32x4 *__restrict__ src,
                                                     f32x4 *__restrict__ dst, int64_t nvec)
{
    const int64_t first = static_cast<int64_t>(blockIdx.x) * (kBlock * kUnroll) + threadIdx.x;
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
        const int64_t i = first + u * kBlock;
        if (i < nvec)
            st_nt(ld_nt(src + i), dst + i);
    }
}

__global__ __launch_bounds__(kBlock) void copy_scalar(const float *__restrict__ src,
                                                        float *__restrict__ dst, int64_t n)
{
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kBlock;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x; i < n; i += stride)
        dst[i] = src[i];
}

int scalar_grid(int64_t n)
{
    const int64_t blocks = ffh::cdiv(n, kBlock);
    return static_cast<int>(blocks < 65536 ? blocks : 65536);
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
    bool vec = true;
    for (const void *p : ptrs) {
        if (!ffh::aligned(p, 4))
            return FF_ERR_ALIGN;
        vec = vec && ffh::aligned(p, 16);
    }
    hipStream_t stream = ffh::as_stream(stream_ptr);
    if (vec) {
        const int64_t nvec = n / 4;
        const int64_t done = nvec * 4;
        if (nvec > 0) {
            const int64_t blocks = ffh::cdiv(nvec, kBlock * kUnroll);
            if (blocks > INT32_MAX)
                return FF_ERR_SIZE;
            hipLaunchKernelGGL(ew_vec<Tag>, dim3(static_cast<unsigned>(blocks)), dim3(kBlock), 0,
                               stream, reinterpret_cast<const f32x4 *>(ah),
                               reinterpret_cast<const f32x4 *>(al),
                               reinterpret_cast<const f32x4 *>(bh),
                               reinterpret_cast<const f32x4 *>(bl),
                               reinterpret_cast<f32x4 *>(rh), reinterpret_cast<f32x4 *>(rl),
                               nvec);
        }
        if (done < n)
            hipLaunchKernelGGL(ew_scalar<Tag>, dim3(1), dim3(kBlock), 0, stream, ah + done,
                               al + done, bh + done, bl + done, rh + done, rl + done, n - done);
    } else {
        hipLaunchKernelGGL(ew_scalar<Tag>, dim3(scalar_grid(n)), dim3(kBlock), 0, stream, ah, al,
                           bh, bl, rh, rl, n);
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
    hipStream_t stream = ffh::as_stream(stream_ptr);
    if (ffh::aligned(src, 16) && ffh::aligned(dst, 16)) {
        const int64_t nvec = n / 4, done = nvec * 4;
        if (nvec > 0) {
            const int64_t blocks = ffh::cdiv(nvec, kBlock * kUnroll);
            if (blocks > INT32_MAX)
                return FF_ERR_SIZE;
            hipLaunchKernelGGL(copy_vec, dim3(static_cast<unsigned>(blocks)), dim3(kBlock), 0,
                               stream, reinterpret_cast<const f32x4 *>(src),
                               reinterpret_cast<f32x4 *>(dst), nvec);
        }
        if (done < n)
            hipLaunchKernelGGL(copy_scalar, dim3(1), dim3(kBlock), 0, stream, src + done,
                               dst + done, n - done);
    } else {
        hipLaunchKernelGGL(copy_scalar, dim3(scalar_grid(n)), dim3(kBlock), 0, stream, src, dst,
                           n);
    }
    return ffh::launch_status();
}

} // extern "C"
