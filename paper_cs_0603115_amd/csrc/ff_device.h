// ff_device.h -- float-float device primitives for gfx950.
//
// Each function performs the binary32 operation sequence of its operator,
// nothing more: the translation unit is compiled with -ffp-contract=off
// (and the pragma below), IEEE binary32 denormals and correctly rounded
// division, so every (+), (-), (x), (/) is one rounded VALU instruction.
// The only fused operation is the explicit __builtin_fmaf of TwoProd.
//
// Paper references are to Da Graca & Defour, "Implementation of float-float
// operators on graphics hardware", section 4.1.
#pragma once

#include <hip/hip_runtime.h>

#pragma clang fp contract(off)

namespace ffd {

// Add12 theorem (Knuth): s = a (+) b, r = (a + b) - s exactly; the
// branch-free six-operation form.
__device__ __forceinline__ void add12(float a, float b, float &s, float &r)
{
    s = a + b;
    const float v = s - a;
    r = (a - (s - v)) + (b - v);
}

// Split theorem (Dekker, after Veltkamp), p = 24 and splitting point 12:
// the product with 2^12 + 1, cancelled against itself, keeps the upper 12
// significant bits of a; the remainder fits in the lower 12 and is exact.
__device__ __forceinline__ void split(float a, float &hi, float &lo)
{
    const float scaled = 4097.0f * a;
    hi = scaled - (scaled - a);
    lo = a - hi;
}

// Mul12 theorem (Dekker's exact product): the four products of the halves
// are exact, so removing three of them from the rounded product x, largest
// first, leaves minus the rounding error exactly; the fourth gives y.
__device__ __forceinline__ void mul12_dekker(float a, float b, float &x, float &y)
{
    x = a * b;
    float a1, a2, b1, b2;
    split(a, a1, a2);
    split(b, b1, b2);
    float rem = x - (a1 * b1);
    rem = rem - (a2 * b1);
    rem = rem - (a1 * b2);
    y = (a2 * b2) - rem;
}

// TwoProd with one fused multiply-add (v_fma_f32): the same pair as Mul12
// whenever the error word is representable.
__device__ __forceinline__ void mul12_fma(float a, float b, float &x, float &y)
{
    x = a * b;
    y = __builtin_fmaf(a, b, -x);
}

// Add22 theorem.  The paper's branch on |ah| >= |bh| is taken as a select
// of which operand plays "a": both arms then evaluate the same chain
// (((x_h (-) r) (+) y_h) (+) y_l) (+) x_l, which is the printed expression
// of the arm selected, so the bits are those of the branching form.
__device__ __forceinline__ void add22(float ah, float al, float bh, float bl,
                                      float &rh, float &rl)
{
    const float r = ah + bh;
    const bool a_big = __builtin_fabsf(ah) >= __builtin_fabsf(bh);
    const float xh = a_big ? ah : bh;
    const float xl = a_big ? al : bl;
    const float yh = a_big ? bh : ah;
    const float yl = a_big ? bl : al;
    const float s = (((xh - r) + yh) + yl) + xl;
    add12(r, s, rh, rl);
}

// Fast2Sum: s = a (+) b and r = b (-) (s (-) a), exact when |a| >= |b|.
__device__ __forceinline__ void fast_add12(float a, float b, float &s, float &r)
{
    s = a + b;
    const float z = s - a;
    r = b - z;
}

// Cancellation-safe addition (not in the paper: its Add22 bound is not
// relative when the operands cancel).  Joldes, Muller and Popescu's
// AccurateDWPlusDW (ACM TOMS 2017): the high and the low words are added
// with exact TwoSums, the low sum is folded into the high one, and two
// Fast2Sums renormalise; relative error below 3u^2/(1 - 4u), u = 2^-24.
__device__ __forceinline__ void add22_accurate(float ah, float al, float bh, float bl,
                                               float &rh, float &rl)
{
    float sh, sl, th, tl, vh, vl;
    add12(ah, bh, sh, sl);
    add12(al, bl, th, tl);
    const float c = sl + th;
    fast_add12(sh, c, vh, vl);
    const float w = tl + vl;
    fast_add12(vh, w, rh, rl);
}

// Mul22 theorem with final step Add12(t1, t3).
template <bool DEKKER>
__device__ __forceinline__ void mul22(float ah, float al, float bh, float bl,
                                      float &rh, float &rl)
{
    float t1, t2;
    if (DEKKER)
        mul12_dekker(ah, bh, t1, t2);
    else
        mul12_fma(ah, bh, t1, t2);
    const float t3 = ((ah * bl) + (al * bh)) + t2;
    add12(t1, t3, rh, rl);
}

// Div22 after Dekker's div2 (the paper has no division).
__device__ __forceinline__ void div22(float ah, float al, float bh, float bl,
                                      float &rh, float &rl)
{
    const float c = ah / bh;
    float u, uu;
    mul12_fma(c, bh, u, uu);
    const float t = (((ah - u) - uu) + al) - (c * bl);
    const float cc = t / bh;
    add12(c, cc, rh, rl);
}

// FMA-based product (not in the paper; its Mul22 bound is 2^-44 = 16u^2):
// Joldes, Muller and Popescu's DWTimesDW3 (ACM TOMS 2017).  The three cross
// products enter through two fused multiply-adds, smallest first, and one
// Fast2Sum renormalises; relative error at most 5u^2, u = 2^-24.
__device__ __forceinline__ void mul22_accurate(float ah, float al, float bh, float bl,
                                               float &rh, float &rl)
{
    float ch, cl1;
    mul12_fma(ah, bh, ch, cl1);
    const float tl0 = al * bl;
    const float tl1 = __builtin_fmaf(ah, bl, tl0);
    const float cl2 = __builtin_fmaf(al, bh, tl1);
    const float cl3 = cl1 + cl2;
    fast_add12(ch, cl3, rh, rl);
}

// Reciprocal-based division (not in the paper): Joldes, Muller and
// Popescu's DWDivDW3 (ACM TOMS 2017), relative error at most 9.8u^2.
// th = 1/bh is refined by one Newton step into a float-float reciprocal m of
// b: the residual e = 1 - b*th (its high part exact by one fma) times th,
// plus th; the quotient is the product a*m above.  The residual's two words
// are joined by the six-operation TwoSum, exact in either order of magnitude.
// Valid for 2^-126 < |bh| < 2^126, where 1/bh is a normal number.
__device__ __forceinline__ void div22_accurate(float ah, float al, float bh, float bl,
                                               float &rh, float &rl)
{
    const float th = 1.0f / bh;
    const float eh0 = __builtin_fmaf(-bh, th, 1.0f);
    const float el0 = -bl * th;
    float eh, el;
    add12(eh0, el0, eh, el);
    float dh, dl1;
    mul12_fma(eh, th, dh, dl1);                 // (eh, el) * th ...
    const float dl = __builtin_fmaf(el, th, dl1);
    float dh2, dl2;
    fast_add12(dh, dl, dh2, dl2);
    float sh, sl;
    add12(dh2, th, sh, sl);                     // ... + th
    const float v = dl2 + sl;
    float mh, ml;
    fast_add12(sh, v, mh, ml);
    mul22_accurate(ah, al, mh, ml, rh, rl);
}

// Butterfly all-reduce of a float-float value over the 64 lanes of a
// wavefront: at distance m = 32, 16, ..., 1 every lane adds its partner's
// value with Add22.  Add22 is commutative bit for bit (swapping the operands
// swaps which one the select calls "a" and leaves the chain unchanged), so
// partners compute identical sums and every lane ends with the same bits.
__device__ __forceinline__ void wave_allreduce_add22(float &h, float &l)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        const float oh = __shfl_xor(h, m, 64);
        const float ol = __shfl_xor(l, m, 64);
        add22(h, l, oh, ol, h, l);
    }
}

// Operator codes shared by the elementwise kernels and the C ABI.
enum Op : int {
    OP_ADD = 0,
    OP_SUB = 1,
    OP_MUL = 2,
    OP_MUL_DEKKER = 3,
    OP_DIV = 4,
    OP_ADD_ACCURATE = 5,
    OP_SUB_ACCURATE = 6,
    OP_MUL_ACCURATE = 7,
    OP_DIV_ACCURATE = 8
};

template <int OP>
__device__ __forceinline__ void apply(float ah, float al, float bh, float bl,
                                      float &rh, float &rl)
{
    if constexpr (OP == OP_ADD)
        add22(ah, al, bh, bl, rh, rl);
    else if constexpr (OP == OP_SUB)
        add22(ah, al, -bh, -bl, rh, rl);
    else if constexpr (OP == OP_MUL)
        mul22<false>(ah, al, bh, bl, rh, rl);
    else if constexpr (OP == OP_MUL_DEKKER)
        mul22<true>(ah, al, bh, bl, rh, rl);
    else if constexpr (OP == OP_DIV)
        div22(ah, al, bh, bl, rh, rl);
    else if constexpr (OP == OP_ADD_ACCURATE)
        add22_accurate(ah, al, bh, bl, rh, rl);
    else if constexpr (OP == OP_SUB_ACCURATE)
        add22_accurate(ah, al, -bh, -bl, rh, rl);
    else if constexpr (OP == OP_MUL_ACCURATE)
        mul22_accurate(ah, al, bh, bl, rh, rl);
    else
        div22_accurate(ah, al, bh, bl, rh, rl);
}

} // namespace ffd
