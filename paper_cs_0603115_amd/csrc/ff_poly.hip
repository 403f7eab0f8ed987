// ff_poly.hip -- polynomial evaluation at many points: Horner's rule in
// binary32, compensated Horner and float-float Horner.
//
// Compensated algorithms are the paper's stated future work (section 7).
// CompHorner (Graillat, Langlois and Louvet, 2005) runs Horner's rule in
// binary32 and catches both rounding errors of every step with error-free
// transforms (TwoProd, then TwoSum, section 4.1), accumulating them by a
// second Horner recurrence; the result is as accurate as Horner's rule in
// twice the working precision, rounded once.  Float-float Horner evaluates
// with the paper's Mul22 and Add22 and returns a float-float value.
//
// Data: p(x) = sum_{i=0..degree} c[i] x^i, coefficients ascending in device
// memory (float-float: two planes), one result per point; points and results
// are SoA planes.  Every lane evaluates four consecutive points (one float4
// of every plane), four independent recurrences that keep the VALU busy; the
// coefficient index is the same in every lane, so coefficients arrive
// through scalar loads and cost no vector memory traffic.
//
// Cost per point and degree: 2 floating-point operations (Horner), 11
// (CompHorner: TwoProd 2, TwoSum 6, correction 3), 23 (Mul22 12 + Add22 11,
// plus Add22's compare-and-select); 8 bytes of memory per point for the
// binary32 forms, 12 for float-float Horner at binary32 points.  Against
// gfx950's ridge of ~9.8 binary32 operations per byte, binary32 Horner stays
// HBM-bound up to degree ~39, while CompHorner (above degree ~7) and
// float-float Horner (above degree ~5) are bound by the VALU.
#include "ff_device.h"
#include "ff_host.h"

namespace ffk {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kPolyBlock = 256;

struct PolyArgs {
    const float *ch;    // coefficients (high words), degree + 1
    const float *cl;    // low words, or null (zeros)
    int32_t degree;
    const float *xh;    // points (high words)
    const float *xl;    // low words, or null (zeros)
    float *yh;          // results (the single result word of the binary32 forms)
    float *yl;          // low words of the float-float result, else unused
};

// Horner's rule in binary32: s = (s (x) x) (+) c_i, two roundings per step.
struct HornerF32 {
    static constexpr bool kFF = false;
    struct State { float s; };
    __device__ __forceinline__ static void init(State &st, float ch, float) { st.s = ch; }
    __device__ __forceinline__ static void step(State &st, float x, float, float ch, float)
    {
        st.s = (st.s * x) + ch;
    }
    __device__ __forceinline__ static void result(const State &st, float &yh, float &)
    {
        yh = st.s;
    }
};

// CompHorner: (p, pi) = TwoProd(s, x); (s, sigma) = TwoSum(p, c_i);
// r = (r (x) x) (+) (pi (+) sigma); result s (+) r.
struct HornerComp {
    static constexpr bool kFF = false;
    struct State { float s, r; };
    __device__ __forceinline__ static void init(State &st, float ch, float)
    {
        st.s = ch;
        st.r = 0.0f;
    }
    __device__ __forceinline__ static void step(State &st, float x, float, float ch, float)
    {
        float p, pi, sigma;
        ffd::mul12_fma(st.s, x, p, pi);
        ffd::add12(p, ch, st.s, sigma);
        st.r = (st.r * x) + (pi + sigma);
    }
    __device__ __forceinline__ static void result(const State &st, float &yh, float &)
    {
        yh = st.s + st.r;
    }
};

// Float-float Horner: s = Add22(Mul22(s, x), c_i).
struct HornerFF {
    static constexpr bool kFF = true;
    struct State { float h, l; };
    __device__ __forceinline__ static void init(State &st, float ch, float cl)
    {
        st.h = ch;
        st.l = cl;
    }
    __device__ __forceinline__ static void step(State &st, float xh, float xl, float ch, float cl)
    {
        float ph, pl;
        ffd::mul22<false>(st.h, st.l, xh, xl, ph, pl);
        ffd::add22(ph, pl, ch, cl, st.h, st.l);
    }
    __device__ __forceinline__ static void result(const State &st, float &yh, float &yl)
    {
        yh = st.h;
        yl = st.l;
    }
};

// Four points per lane: the float4 group g of every plane.
template <class Alg, bool CLO, bool XLO>
__global__ __launch_bounds__(kPolyBlock) void horner_vec(PolyArgs a, int64_t ngroups)
{
    const int64_t g = static_cast<int64_t>(blockIdx.x) * kPolyBlock + threadIdx.x;
    if (g >= ngroups)
        return;
    const f32x4 xh = __builtin_nontemporal_load(reinterpret_cast<const f32x4 *>(a.xh) + g);
    f32x4 xl = {0.0f, 0.0f, 0.0f, 0.0f};
    if constexpr (XLO)
        xl = __builtin_nontemporal_load(reinterpret_cast<const f32x4 *>(a.xl) + g);
    typename Alg::State st[4];
    {
        const float th = a.ch[a.degree];
        const float tl = CLO ? a.cl[a.degree] : 0.0f;
#pragma unroll
        for (int c = 0; c < 4; ++c)
            Alg::init(st[c], th, tl);
    }
#pragma unroll 4
    for (int32_t i = a.degree - 1; i >= 0; --i) {
        const float ch = a.ch[i];
        const float cl = CLO ? a.cl[i] : 0.0f;
#pragma unroll
        for (int c = 0; c < 4; ++c)
            Alg::step(st[c], xh[c], xl[c], ch, cl);
    }
    f32x4 yh, yl;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        float h, l = 0.0f;
        Alg::result(st[c], h, l);
        yh[c] = h;
        yl[c] = l;
    }
    __builtin_nontemporal_store(yh, reinterpret_cast<f32x4 *>(a.yh) + g);
    if constexpr (Alg::kFF)
        __builtin_nontemporal_store(yl, reinterpret_cast<f32x4 *>(a.yl) + g);
}

// One point per lane: the tail after the float4 groups, and planes that are
// not 16-byte aligned.
template <class Alg, bool CLO, bool XLO>
__global__ __launch_bounds__(kPolyBlock) void horner_scalar(PolyArgs a, int64_t n)
{
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kPolyBlock;
    for (int64_t k = static_cast<int64_t>(blockIdx.x) * kPolyBlock + threadIdx.x; k < n;
         k += stride) {
        const float xh = a.xh[k];
        const float xl = XLO ? a.xl[k] : 0.0f;
        typename Alg::State st;
        Alg::init(st, a.ch[a.degree], CLO ? a.cl[a.degree] : 0.0f);
        for (int32_t i = a.degree - 1; i >= 0; --i)
            Alg::step(st, xh, xl, a.ch[i], CLO ? a.cl[i] : 0.0f);
        float h, l = 0.0f;
        Alg::result(st, h, l);
        a.yh[k] = h;
        if constexpr (Alg::kFF)
            a.yl[k] = l;
    }
}

template <class Alg, bool CLO, bool XLO>
ff_status launch_horner(PolyArgs a, int64_t n, bool vec, hipStream_t st)
{
    int64_t done = 0;
    if (vec) {
        const int64_t ngroups = n / 4;
        done = 4 * ngroups;
        if (ngroups > 0) {
            const int64_t blocks = ffh::cdiv(ngroups, kPolyBlock);
            if (blocks > INT32_MAX)
                return FF_ERR_SIZE;
            hipLaunchKernelGGL((horner_vec<Alg, CLO, XLO>), dim3(static_cast<unsigned>(blocks)),
                               dim3(kPolyBlock), 0, st, a, ngroups);
        }
    }
    if (done < n) {
        PolyArgs rest = a;
        rest.xh += done;
        if (XLO)
            rest.xl += done;
        rest.yh += done;
        if (Alg::kFF)
            rest.yl += done;
        const int64_t blocks = ffh::cdiv(n - done, kPolyBlock);
        hipLaunchKernelGGL((horner_scalar<Alg, CLO, XLO>),
                           dim3(static_cast<unsigned>(blocks < 65536 ? blocks : 65536)),
                           dim3(kPolyBlock), 0, st, rest, n - done);
    }
    return ffh::launch_status();
}

// Argument checks, then the launch variant for the null-able low words.
template <class Alg>
ff_status horner(PolyArgs a, int64_t n, void *stream_ptr)
{
    if (a.degree < 0 || n < 0)
        return FF_ERR_SIZE;
    if (n == 0)
        return FF_OK;
    if (!a.ch || !a.xh || !a.yh || (Alg::kFF && !a.yl))
        return FF_ERR_NULL;
    const void *planes[] = {a.ch, a.cl, a.xh, a.xl, a.yh, Alg::kFF ? a.yl : nullptr};
    bool vec = true;
    for (const void *p : planes) {
        if (!p)
            continue;
        if (!ffh::aligned(p, 4))
            return FF_ERR_ALIGN;
        if (p != a.ch && p != a.cl)
            vec = vec && ffh::aligned(p, 16);
    }
    hipStream_t st = ffh::as_stream(stream_ptr);
    if constexpr (!Alg::kFF)
        return launch_horner<Alg, false, false>(a, n, vec, st);
    const bool clo = a.cl != nullptr, xlo = a.xl != nullptr;
    if (clo && xlo)
        return launch_horner<Alg, true, true>(a, n, vec, st);
    if (clo)
        return launch_horner<Alg, true, false>(a, n, vec, st);
    if (xlo)
        return launch_horner<Alg, false, true>(a, n, vec, st);
    return launch_horner<Alg, false, false>(a, n, vec, st);
}

} // namespace ffk

using namespace ffk;

extern "C" {

ff_status ff_horner_f32(const float *coef, int32_t degree, const float *x, float *y, int64_t n,
                        void *stream)
{
    return horner<HornerF32>(PolyArgs{coef, nullptr, degree, x, nullptr, y, nullptr}, n, stream);
}

ff_status ff_horner_comp(const float *coef, int32_t degree, const float *x, float *y, int64_t n,
                         void *stream)
{
    return horner<HornerComp>(PolyArgs{coef, nullptr, degree, x, nullptr, y, nullptr}, n, stream);
}

ff_status ff_horner_ff(const float *coef_hi, const float *coef_lo, int32_t degree,
                       const float *x_hi, const float *x_lo, float *y_hi, float *y_lo, int64_t n,
                       void *stream)
{
    return horner<HornerFF>(PolyArgs{coef_hi, coef_lo, degree, x_hi, x_lo, y_hi, y_lo}, n,
                            stream);
}

} // extern "C"
