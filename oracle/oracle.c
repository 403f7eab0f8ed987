/*
 * Float-float reference oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, scalar CPU implementation of the float-float operators of
 * Da Graca & Defour, "Implementation of float-float operators on graphics
 * hardware" (cs/0603115).  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library; the product path
 * (the HIP library) never does, and the two share no code.
 *
 * Arithmetic model.  Every operation written below as a C float operation is
 * ONE IEEE-754 binary32 operation rounded to nearest-even: this file must be
 * built with SSE floating point (x86-64 default, FLT_EVAL_METHOD == 0),
 * -ffp-contract=off and without -ffast-math, and runs with the default MXCSR
 * (subnormals neither flushed nor treated as zero).  The paper writes these
 * rounded operations as (+), (-), (x), (/) (section 4.1); its proofs assume
 * faithful rounding with a guard bit, which round-to-nearest satisfies.
 * The only fused operation is fmaf(), used solely by the FMA form of TwoProd.
 *
 * Readings of the paper taken here (each one is listed in the design notes):
 *   - Add12 everywhere is the branch-free six-operation form (section 4
 *     prefers it; section 4.1, Add12 theorem).
 *   - Mul22's final step renormalises (t1, t3): the printed Add12(t1, t2)
 *     leaves t3 unused, a typo (section 4.1, Mul22 theorem).
 *   - Division is not defined by the paper: Div22 follows Dekker's div2
 *     (Dekker 1971, the paper's reference for Split and Mul12), with a
 *     correctly rounded binary32 quotient and Add12 as the final step.
 *   - Reductions accumulate exact products with Add22, in index order.
 *
 * Exact references (dot products, GEMM entries, gradients) do not round at
 * all: a long fixed-point accumulator adds every exact FP32xFP32 product.
 *
 * Parity pins: every function here is checked by the CPU test-suite against
 * exact rational arithmetic, closed forms or the paper's error bounds; see the
 * per-function comments.
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#if !defined(FLT_EVAL_METHOD) || FLT_EVAL_METHOD != 0
#error "the oracle needs binary32 evaluation (SSE), not extended precision"
#endif

#pragma STDC FP_CONTRACT OFF

#define ORACLE_ABI_VERSION 1

int oracle_abi_version(void) { return ORACLE_ABI_VERSION; }

/* ------------------------------------------------------------------------ */
/* Error-free transformations (section 4.1)                                 */
/* ------------------------------------------------------------------------ */

/* Add12 theorem (Knuth): s = a (+) b and r with s + r = a + b exactly.
 * Six rounded operations, no branch. */
static void add12(float a, float b, float *s_out, float *r_out)
{
    float s = a + b;
    float v = s - a;
    float r = (a - (s - v)) + (b - v);
    *s_out = s;
    *r_out = r;
}

/* The "one test" Add12 the paper mentions next to the branch-free one
 * (section 4): Fast2Sum, exact when |a| >= |b|.  None of the paper's
 * operators uses it; the cancellation-safe addition below does, where its
 * operands are ordered. */
static void fast_add12(float a, float b, float *s_out, float *r_out)
{
    float s = a + b;
    float z = s - a;
    *s_out = s;
    *r_out = b - z;
}

/* Split theorem (Dekker, after Veltkamp): for p = 24 and the splitting
 * point 12, scaling by 2^12 + 1 and cancelling the scaled value against
 * itself leaves the upper 12 significant bits of a; the remainder a - hi
 * then fits in the other 12 bits (sign included) and is exact. */
static void split(float a, float *hi_out, float *lo_out)
{
    const float c_split = 4097.0f; /* 2^12 (+) 1, exact */
    const float scaled = c_split * a;
    const float hi = scaled - (scaled - a);
    *hi_out = hi;
    *lo_out = a - hi;
}

/* Mul12 theorem (Dekker's exact product): with a and b split in halves,
 * the four half products are exact, so peeling them off the rounded product
 * x one by one (largest first) leaves the rounding error -y exactly; the
 * last half product then gives y with a*b = x + y. */
static void mul12_dekker(float a, float b, float *x_out, float *y_out)
{
    const float x = a * b;
    float a1, a2, b1, b2; /* a = a1 + a2, b = b1 + b2, 12 bits each */
    split(a, &a1, &a2);
    split(b, &b1, &b2);
    float rem = x - (a1 * b1);
    rem = rem - (a2 * b1);
    rem = rem - (a1 * b2);
    *x_out = x;
    *y_out = (a2 * b2) - rem;
}

/* TwoProd with one fused multiply-add (not in the paper; same contract as
 * Mul12): y = fma(a, b, -x) is the exact error of x = a (x) b whenever that
 * error is representable. */
static void mul12_fma(float a, float b, float *x_out, float *y_out)
{
    float x = a * b;
    *x_out = x;
    *y_out = fmaf(a, b, -x);
}

static void mul12(float a, float b, int use_dekker, float *x, float *y)
{
    if (use_dekker)
        mul12_dekker(a, b, x, y);
    else
        mul12_fma(a, b, x, y);
}

/* ------------------------------------------------------------------------ */
/* Float-float operators (section 4.1, Add22 and Mul22 theorems; Div22 from   */
/* Dekker's div2)                                                            */
/* ------------------------------------------------------------------------ */

/* Add22 theorem: the sum of two float-float numbers, branch on |ah| >= |bh|,
 * each chain evaluated left to right as parenthesised in the paper. */
static void add22(float ah, float al, float bh, float bl, float *rh, float *rl)
{
    float r = ah + bh;
    float s;
    if (fabsf(ah) >= fabsf(bh))
        s = (((ah - r) + bh) + bl) + al;
    else
        s = (((bh - r) + ah) + al) + bl;
    add12(r, s, rh, rl);
}

/* Sub22: Add22 with the second operand negated (negation is exact). */
static void sub22(float ah, float al, float bh, float bl, float *rh, float *rl)
{
    add22(ah, al, -bh, -bl, rh, rl);
}

/* Cancellation-safe float-float addition (not in the paper, whose Add22
 * bound is not relative under cancellation, Add22 theorem): the
 * "AccurateDWPlusDW" algorithm of Joldes, Muller and Popescu (ACM TOMS 2017,
 * Algorithm 6), relative error below 3u^2 / (1 - 4u), u = 2^-24:
 *   (sh, sl) = TwoSum(ah, bh);  (th, tl) = TwoSum(al, bl);
 *   c = sl + th;  (vh, vl) = Fast2Sum(sh, c);  w = tl + vl;
 *   (rh, rl) = Fast2Sum(vh, w). */
static void add22_accurate(float ah, float al, float bh, float bl, float *rh,
                           float *rl)
{
    float sh, sl, th, tl, vh, vl;
    add12(ah, bh, &sh, &sl);
    add12(al, bl, &th, &tl);
    float c = sl + th;
    fast_add12(sh, c, &vh, &vl);
    float w = tl + vl;
    fast_add12(vh, w, rh, rl);
}

/* FMA-based float-float product (not in the paper; a tighter-bound
 * alternative to Mul22): the "DWTimesDW3" algorithm of Joldes, Muller and
 * Popescu (ACM TOMS 2017, Algorithm 12), relative error at most 5u^2,
 * u = 2^-24:
 *   (ch, cl1) = TwoProd(ah, bh);  tl0 = al * bl;  tl1 = fma(ah, bl, tl0);
 *   cl2 = fma(al, bh, tl1);  cl3 = cl1 + cl2;  (rh, rl) = Fast2Sum(ch, cl3).
 * Fast2Sum is exact here: |cl3| is below ulp(ch) for normalised inputs. */
static void mul22_accurate(float ah, float al, float bh, float bl, float *rh,
                           float *rl)
{
    float ch, cl1;
    mul12_fma(ah, bh, &ch, &cl1);
    float tl0 = al * bl;
    float tl1 = fmaf(ah, bl, tl0);
    float cl2 = fmaf(al, bh, tl1);
    float cl3 = cl1 + cl2;
    fast_add12(ch, cl3, rh, rl);
}

/* Reciprocal-based float-float division (not in the paper): the "DWDivDW3"
 * algorithm of Joldes, Muller and Popescu (ACM TOMS 2017, Algorithm 18),
 * relative error at most 9.8u^2.  One Newton step refines th = 1/bh into a
 * float-float reciprocal m of b, and the quotient is the product a * m:
 *   th = 1 / bh;  rh = fma(-bh, th, 1) (exact);  rl = -bl * th;
 *   (eh, el) = TwoSum(rh, rl);
 *   (dh, dl) = (eh, el) * th         [DWTimesFP3: TwoProd(eh, th),
 *                                      fma(el, th, error), Fast2Sum];
 *   (mh, ml) = (dh, dl) + th         [DWPlusFP: TwoSum(dh, th), add the
 *                                      low words, Fast2Sum];
 *   (rh, rl) = a * m                 [DWTimesDW3 above].
 * (eh, el) uses the six-operation TwoSum: |rl| may exceed |rh|, and TwoSum
 * is exact for any order (equal to Fast2Sum wherever that one is exact).
 * Valid for 2^-126 < |bh| < 2^126, where 1/bh is a normal number. */
static void div22_accurate(float ah, float al, float bh, float bl, float *rh,
                           float *rl)
{
    float th = 1.0f / bh;
    float eh0 = fmaf(-bh, th, 1.0f);
    float el0 = -bl * th;
    float eh, el;
    add12(eh0, el0, &eh, &el);
    float dh, dl1;
    mul12_fma(eh, th, &dh, &dl1);
    float dl = fmaf(el, th, dl1);
    float dh2, dl2;
    fast_add12(dh, dl, &dh2, &dl2);
    float sh, sl;
    add12(dh2, th, &sh, &sl);
    float v = dl2 + sl;
    float mh, ml;
    fast_add12(sh, v, &mh, &ml);
    mul22_accurate(ah, al, mh, ml, rh, rl);
}

/* Mul22 theorem, with the final renormalisation of (t1, t3). */
static void mul22(float ah, float al, float bh, float bl, int use_dekker,
                  float *rh, float *rl)
{
    float t1, t2;
    mul12(ah, bh, use_dekker, &t1, &t2);
    float t3 = ((ah * bl) + (al * bh)) + t2;
    add12(t1, t3, rh, rl);
}

/* Div22 after Dekker's div2: c = ah / bh; (u, uu) = c * bh exactly;
 * cc = ((((ah - u) - uu) + al) - c*bl) / bh; result = Add12(c, cc). */
static void div22(float ah, float al, float bh, float bl, int use_dekker,
                  float *rh, float *rl)
{
    float c = ah / bh;
    float u, uu;
    mul12(c, bh, use_dekker, &u, &uu);
    float t = (((ah - u) - uu) + al) - (c * bl);
    float cc = t / bh;
    add12(c, cc, rh, rl);
}

/* ------------------------------------------------------------------------ */
/* Array entry points: one scalar loop each, element i independent.         */
/* ------------------------------------------------------------------------ */

void oracle_add12(const float *a, const float *b, float *s, float *r, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        add12(a[i], b[i], &s[i], &r[i]);
}

void oracle_fast_add12(const float *a, const float *b, float *s, float *r,
                       int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        fast_add12(a[i], b[i], &s[i], &r[i]);
}

void oracle_split(const float *a, float *hi, float *lo, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        split(a[i], &hi[i], &lo[i]);
}

void oracle_mul12(const float *a, const float *b, float *x, float *y, int64_t n,
                  int use_dekker)
{
    for (int64_t i = 0; i < n; ++i)
        mul12(a[i], b[i], use_dekker, &x[i], &y[i]);
}

void oracle_add22(const float *ah, const float *al, const float *bh,
                  const float *bl, float *rh, float *rl, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        add22(ah[i], al[i], bh[i], bl[i], &rh[i], &rl[i]);
}

void oracle_sub22(const float *ah, const float *al, const float *bh,
                  const float *bl, float *rh, float *rl, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        sub22(ah[i], al[i], bh[i], bl[i], &rh[i], &rl[i]);
}

void oracle_mul22(const float *ah, const float *al, const float *bh,
                  const float *bl, float *rh, float *rl, int64_t n,
                  int use_dekker)
{
    for (int64_t i = 0; i < n; ++i)
        mul22(ah[i], al[i], bh[i], bl[i], use_dekker, &rh[i], &rl[i]);
}

void oracle_div22(const float *ah, const float *al, const float *bh,
                  const float *bl, float *rh, float *rl, int64_t n,
                  int use_dekker)
{
    for (int64_t i = 0; i < n; ++i)
        div22(ah[i], al[i], bh[i], bl[i], use_dekker, &rh[i], &rl[i]);
}

void oracle_mul22_accurate(const float *ah, const float *al, const float *bh,
                           const float *bl, float *rh, float *rl, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        mul22_accurate(ah[i], al[i], bh[i], bl[i], &rh[i], &rl[i]);
}

void oracle_div22_accurate(const float *ah, const float *al, const float *bh,
                           const float *bl, float *rh, float *rl, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        div22_accurate(ah[i], al[i], bh[i], bl[i], &rh[i], &rl[i]);
}

void oracle_add22_accurate(const float *ah, const float *al, const float *bh,
                           const float *bl, float *rh, float *rl, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        add22_accurate(ah[i], al[i], bh[i], bl[i], &rh[i], &rl[i]);
}

void oracle_sub22_accurate(const float *ah, const float *al, const float *bh,
                           const float *bl, float *rh, float *rl, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        add22_accurate(ah[i], al[i], -bh[i], -bl[i], &rh[i], &rl[i]);
}

/* Conversions between binary64 and float-float (not in the paper, whose
 * inputs are float-float already).  From binary64: hi = fl32(x) and
 * lo = fl32(x - hi); x - hi is exact in binary64 (hi is x rounded to 24
 * bits), so hi + lo is x to within 2^-48 |x|, for |x| below the binary32
 * overflow threshold.  To binary64: (double) hi + (double) lo, one binary64
 * rounding (exact whenever the pair's bits fit in 53). */
void oracle_from_f64(const double *x, float *hi, float *lo, int64_t n)
{
    for (int64_t i = 0; i < n; ++i) {
        float h = (float)x[i];
        hi[i] = h;
        lo[i] = (float)(x[i] - (double)h);
    }
}

void oracle_to_f64(const float *hi, const float *lo, double *x, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        x[i] = (double)hi[i] + (double)lo[i];
}

/* Elementwise op selected by code: 0 add, 1 sub, 2 mul (FMA TwoProd),
 * 3 mul (Dekker TwoProd), 4 div (FMA TwoProd), 5 cancellation-safe add,
 * 6 cancellation-safe sub, 7 FMA-based product, 8 reciprocal-based
 * division.  Used by the benchmark's CPU leg so that one call
 * times one operator over a sample. */
int oracle_elementwise(int op, const float *ah, const float *al,
                       const float *bh, const float *bl, float *rh, float *rl,
                       int64_t n)
{
    switch (op) {
    case 0: oracle_add22(ah, al, bh, bl, rh, rl, n); return 0;
    case 1: oracle_sub22(ah, al, bh, bl, rh, rl, n); return 0;
    case 2: oracle_mul22(ah, al, bh, bl, rh, rl, n, 0); return 0;
    case 3: oracle_mul22(ah, al, bh, bl, rh, rl, n, 1); return 0;
    case 4: oracle_div22(ah, al, bh, bl, rh, rl, n, 0); return 0;
    case 5: oracle_add22_accurate(ah, al, bh, bl, rh, rl, n); return 0;
    case 6: oracle_sub22_accurate(ah, al, bh, bl, rh, rl, n); return 0;
    case 7: oracle_mul22_accurate(ah, al, bh, bl, rh, rl, n); return 0;
    case 8: oracle_div22_accurate(ah, al, bh, bl, rh, rl, n); return 0;
    default: return -1;
    }
}

/* Binary32 reference operators, timed beside the float-float ones in the
 * paper's tables (section 6, Tables 3 and 4): 0 add, 1 multiply, 2 multiply-
 * add with a single rounding (fmaf).  Returns -1 for an unknown op. */
int oracle_f32_ref(int op, const float *a, const float *b, const float *c,
                   float *r, int64_t n)
{
    switch (op) {
    case 0:
        for (int64_t i = 0; i < n; ++i)
            r[i] = a[i] + b[i];
        return 0;
    case 1:
        for (int64_t i = 0; i < n; ++i)
            r[i] = a[i] * b[i];
        return 0;
    case 2:
        for (int64_t i = 0; i < n; ++i)
            r[i] = fmaf(a[i], b[i], c[i]);
        return 0;
    default:
        return -1;
    }
}

/* ------------------------------------------------------------------------ */
/* Float-float accumulation in index order (reductions, matvec, plain GEMM) */
/* ------------------------------------------------------------------------ */

/* dot of FP32 vectors: acc = Add22(acc, TwoProd_fma(x_i, y_i)), i ascending. */
void oracle_dot_seq(const float *x, const float *y, int64_t n, float *out2)
{
    float acc_h = 0.0f, acc_l = 0.0f;
    for (int64_t i = 0; i < n; ++i) {
        float p, e;
        mul12_fma(x[i], y[i], &p, &e);
        add22(acc_h, acc_l, p, e, &acc_h, &acc_l);
    }
    out2[0] = acc_h;
    out2[1] = acc_l;
}

/* dot of float-float vectors with strides:
 * acc = Add22(acc, Mul22(x_i, y_i)), i ascending (FMA TwoProd). */
void oracle_dot_ff_seq(const float *xh, const float *xl, int64_t incx,
                       const float *yh, const float *yl, int64_t incy,
                       int64_t n, float *out2)
{
    float acc_h = 0.0f, acc_l = 0.0f;
    for (int64_t i = 0; i < n; ++i) {
        float ph, pl;
        mul22(xh[i * incx], xl[i * incx], yh[i * incy], yl[i * incy], 0, &ph,
              &pl);
        add22(acc_h, acc_l, ph, pl, &acc_h, &acc_l);
    }
    out2[0] = acc_h;
    out2[1] = acc_l;
}

/* Plain float-float GEMM on the block rows [i0,i1) x cols [j0,j1) of
 * C = A*B (row-major): C_ij = Add22-accumulation over k ascending of
 * Mul22(A_ik, B_kj), starting from (0, 0).  The block is stored at
 * C[(i - i0) * ldc + (j - j0)]. */
void oracle_gemm_ff_seq(int64_t K, const float *Ah, const float *Al, int64_t lda,
                        const float *Bh, const float *Bl, int64_t ldb, float *Ch,
                        float *Cl, int64_t ldc, int64_t i0, int64_t i1,
                        int64_t j0, int64_t j1)
{
    for (int64_t i = i0; i < i1; ++i)
        for (int64_t j = j0; j < j1; ++j) {
            float out[2];
            oracle_dot_ff_seq(Ah + i * lda, Al + i * lda, 1, Bh + j, Bl + j,
                              ldb, K, out);
            Ch[(i - i0) * ldc + (j - j0)] = out[0];
            Cl[(i - i0) * ldc + (j - j0)] = out[1];
        }
}

/* ------------------------------------------------------------------------ */
/* Compensated summation and dot product (Ogita, Rump and Oishi 2005)        */
/* ------------------------------------------------------------------------ */
/*
 * The paper names compensated algorithms as future work (section 7).  These
 * are the working-precision algorithms Sum2 and Dot2 of Ogita, Rump and
 * Oishi ("Accurate sum and dot product", SIAM J. Sci. Comput. 26(6), 2005):
 *   Sum2: p = x_1, s = 0; for i >= 2: (p, q) = TwoSum(p, x_i), s = s (+) q;
 *   Dot2: (p, s) = TwoProduct(x_1, y_1); for i >= 2:
 *         (h, r) = TwoProduct(x_i, y_i), (p, q) = TwoSum(p, h),
 *         s = s (+) (q (+) r);
 * the result is p (+) s.  TwoProduct is the FMA form.  out2 receives
 * (p, s), the unevaluated result before its final rounding; n = 0 gives
 * (0, 0).
 */
void oracle_sum2(const float *x, int64_t n, float *out2)
{
    float p = 0.0f, s = 0.0f;
    if (n > 0)
        p = x[0];
    for (int64_t i = 1; i < n; ++i) {
        float q;
        add12(p, x[i], &p, &q);
        s = s + q;
    }
    out2[0] = p;
    out2[1] = s;
}

void oracle_dot2(const float *x, const float *y, int64_t n, float *out2)
{
    float p = 0.0f, s = 0.0f;
    if (n > 0)
        mul12_fma(x[0], y[0], &p, &s);
    for (int64_t i = 1; i < n; ++i) {
        float h, r, q;
        mul12_fma(x[i], y[i], &h, &r);
        add12(p, h, &p, &q);
        s = s + (q + r);
    }
    out2[0] = p;
    out2[1] = s;
}

/* Batched forms over concatenated vectors (vector v is [offsets[v],
 * offsets[v+1])); out2 has 2 * nvec entries. */
void oracle_sum2_batched(const float *x, const int64_t *offsets, int64_t nvec,
                         float *out2)
{
    for (int64_t v = 0; v < nvec; ++v)
        oracle_sum2(x + offsets[v], offsets[v + 1] - offsets[v], out2 + 2 * v);
}

void oracle_dot2_batched(const float *x, const float *y, const int64_t *offsets,
                         int64_t nvec, float *out2)
{
    for (int64_t v = 0; v < nvec; ++v)
        oracle_dot2(x + offsets[v], y + offsets[v], offsets[v + 1] - offsets[v],
                    out2 + 2 * v);
}

/* ------------------------------------------------------------------------ */
/* Polynomial evaluation: Horner's rule in binary32, compensated Horner,     */
/* float-float Horner                                                        */
/* ------------------------------------------------------------------------ */
/*
 * p(x) = sum_{i=0..degree} a[i] x^i, coefficients in ascending order, one
 * evaluation per point.  Compensated algorithms are the paper's stated
 * future work (section 7); CompHorner is that of Graillat, Langlois and
 * Louvet ("Compensated Horner scheme", 2005; "Algorithms for accurate,
 * validated and fast polynomial evaluation", 2009).
 */

/* Horner's rule: s = a_n; s = (s (x) x) (+) a_i for i = n-1 .. 0.  Two
 * roundings per step (no fused multiply-add). */
void oracle_horner_f32(const float *a, int32_t degree, const float *x,
                       float *y, int64_t n)
{
    for (int64_t k = 0; k < n; ++k) {
        float s = a[degree];
        for (int32_t i = degree - 1; i >= 0; --i)
            s = (s * x[k]) + a[i];
        y[k] = s;
    }
}

/* CompHorner: Horner's rule with both rounding errors of every step caught
 * by error-free transforms, (p, pi) = TwoProd(s, x) and
 * (s, sigma) = TwoSum(p, a_i), and accumulated by a second Horner recurrence
 * r = (r (x) x) (+) (pi (+) sigma), r_n = 0; the result is s_0 (+) r_0.
 * Its error is at most u |p(x)| + gamma_2n^2 sum |a_i| |x|^i (u = 2^-24,
 * gamma_k = k u / (1 - k u)) without underflow. */
void oracle_horner_comp(const float *a, int32_t degree, const float *x,
                        float *y, int64_t n)
{
    for (int64_t k = 0; k < n; ++k) {
        const float xk = x[k];
        float s = a[degree];
        float r = 0.0f;
        for (int32_t i = degree - 1; i >= 0; --i) {
            float p, pi, sigma;
            mul12_fma(s, xk, &p, &pi);
            add12(p, a[i], &s, &sigma);
            r = (r * xk) + (pi + sigma);
        }
        y[k] = s + r;
    }
}

/* Float-float Horner: s = a_n; s = Add22(Mul22(s, x), a_i), coefficients
 * and points as float-float numbers (the paper's Add22 and Mul22 with FMA
 * TwoProd, section 4.1). */
void oracle_horner_ff(const float *ah, const float *al, int32_t degree,
                      const float *xh, const float *xl, float *yh, float *yl,
                      int64_t n)
{
    for (int64_t k = 0; k < n; ++k) {
        float sh = ah[degree], sl = al[degree];
        for (int32_t i = degree - 1; i >= 0; --i) {
            float ph, pl;
            mul22(sh, sl, xh[k], xl[k], 0, &ph, &pl);
            add22(ph, pl, ah[i], al[i], &sh, &sl);
        }
        yh[k] = sh;
        yl[k] = sl;
    }
}

/* Backward pass of the batched float-float dot s_v = sum over vector v of
 * x_i y_i, for upstream float-float gradients g_v: every element i of vector
 * v gets dx_i = Mul22(g_v, y_i) and dy_i = Mul22(g_v, x_i) (FMA TwoProd);
 * elements of no vector get zero gradients.  Offsets non-decreasing, within
 * [0, total]. */
void oracle_dot_batched_backward(const float *gh, const float *gl,
                                 const int64_t *offsets, int64_t nvec,
                                 int64_t total, const float *xh,
                                 const float *xl, const float *yh,
                                 const float *yl, float *dxh, float *dxl,
                                 float *dyh, float *dyl)
{
    for (int64_t i = 0; i < total; ++i)
        dxh[i] = dxl[i] = dyh[i] = dyl[i] = 0.0f;
    for (int64_t v = 0; v < nvec; ++v) {
        for (int64_t i = offsets[v]; i < offsets[v + 1]; ++i) {
            mul22(gh[v], gl[v], yh[i], yl[i], 0, &dxh[i], &dxl[i]);
            mul22(gh[v], gl[v], xh[i], xl[i], 0, &dyh[i], &dyl[i]);
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Exact accumulation: a long fixed-point accumulator                       */
/* ------------------------------------------------------------------------ */
/*
 * Every finite binary32 value is M * 2^E with M an integer, |M| < 2^24, and
 * E >= -149; a product of two is M1*M2 * 2^(E1+E2), |M1*M2| < 2^48,
 * E1+E2 >= -298.  The accumulator holds sum(value) / 2^LA_EMIN as an integer
 * in base-2^32 limbs; each limb is a signed 64-bit word so that it can absorb
 * 2^31 additions of 32-bit pieces before carries must be propagated.
 */
#define LA_LIMBS 24
#define LA_EMIN (-384) /* weight of bit 0 of limb 0 */

int oracle_exact_limbs(void) { return LA_LIMBS; }
int oracle_exact_emin(void) { return LA_EMIN; }

typedef struct {
    int64_t limb[LA_LIMBS];
    int64_t pending; /* additions since the last carry propagation */
} long_acc;

static void la_normalise(long_acc *acc)
{
    for (int i = 0; i < LA_LIMBS - 1; ++i) {
        int64_t carry = acc->limb[i] >> 32; /* floor division by 2^32 */
        acc->limb[i] -= carry * ((int64_t)1 << 32);
        acc->limb[i + 1] += carry;
    }
    acc->pending = 0;
}

/* binary32 -> (M, E) with value = M * 2^E exactly (zero gives M = 0). */
static void f32_decompose(float v, int64_t *m, int *e)
{
    if (v == 0.0f) {
        *m = 0;
        *e = 0;
        return;
    }
    int ex;
    float frac = frexpf(v, &ex); /* v = frac * 2^ex, 0.5 <= |frac| < 1 */
    *m = (int64_t)ldexpf(frac, 24); /* exact: frac has at most 24 bits */
    *e = ex - 24;
}

/* acc += m * 2^e, |m| < 2^62, e >= LA_EMIN. */
static void la_add_scaled(long_acc *acc, int64_t m, int e)
{
    if (m == 0)
        return;
    int pos = e - LA_EMIN;
    int neg = m < 0;
    unsigned __int128 mag = (unsigned __int128)(neg ? -(uint64_t)m : (uint64_t)m);
    mag <<= (pos % 32);
    int li = pos / 32;
    for (int k = 0; k < 4 && mag != 0; ++k) {
        int64_t piece = (int64_t)(uint32_t)(mag & 0xffffffffu);
        acc->limb[li + k] += neg ? -piece : piece;
        mag >>= 32;
    }
    if (++acc->pending >= ((int64_t)1 << 30))
        la_normalise(acc);
}

static void la_add_product(long_acc *acc, float a, float b)
{
    int64_t ma, mb;
    int ea, eb;
    f32_decompose(a, &ma, &ea);
    f32_decompose(b, &mb, &eb);
    la_add_scaled(acc, ma * mb, ea + eb);
}

static void la_store(long_acc *acc, int64_t *limbs_out)
{
    la_normalise(acc);
    memcpy(limbs_out, acc->limb, sizeof(acc->limb));
}

/* Exact sum_i x_i*y_i (FP32 inputs, strided).  limbs_out[LA_LIMBS] receives
 * the result as sum_k limbs_out[k] * 2^(32k + LA_EMIN); every limb but the
 * last lies in [0, 2^32), the last carries the sign. */
void oracle_exact_dot(const float *x, int64_t incx, const float *y,
                      int64_t incy, int64_t n, int64_t *limbs_out)
{
    long_acc acc;
    memset(&acc, 0, sizeof(acc));
    for (int64_t i = 0; i < n; ++i)
        la_add_product(&acc, x[i * incx], y[i * incy]);
    la_store(&acc, limbs_out);
}

/* Exact sum_i (xh_i + xl_i) * (yh_i + yl_i) (float-float inputs, strided). */
void oracle_exact_dot_ff(const float *xh, const float *xl, int64_t incx,
                         const float *yh, const float *yl, int64_t incy,
                         int64_t n, int64_t *limbs_out)
{
    long_acc acc;
    memset(&acc, 0, sizeof(acc));
    for (int64_t i = 0; i < n; ++i) {
        float a = xh[i * incx], al = xl[i * incx];
        float b = yh[i * incy], bl = yl[i * incy];
        la_add_product(&acc, a, b);
        la_add_product(&acc, a, bl);
        la_add_product(&acc, al, b);
        la_add_product(&acc, al, bl);
    }
    la_store(&acc, limbs_out);
}

/* Batched exact dots over concatenated FP32 vectors: vector v occupies
 * [offsets[v], offsets[v+1]).  limbs_out has nvec * LA_LIMBS entries. */
void oracle_exact_dot_batched(const float *x, const float *y,
                              const int64_t *offsets, int64_t nvec,
                              int64_t *limbs_out)
{
    for (int64_t v = 0; v < nvec; ++v)
        oracle_exact_dot(x + offsets[v], 1, y + offsets[v], 1,
                         offsets[v + 1] - offsets[v], limbs_out + v * LA_LIMBS);
}

/* Sequential float-float dots over concatenated FP32 vectors (the CPU
 * baseline of the batched reduction): out2 has 2 * nvec entries. */
void oracle_dot_seq_batched(const float *x, const float *y,
                            const int64_t *offsets, int64_t nvec, float *out2)
{
    for (int64_t v = 0; v < nvec; ++v)
        oracle_dot_seq(x + offsets[v], y + offsets[v],
                       offsets[v + 1] - offsets[v], out2 + 2 * v);
}

/* Exact GEMM entries C_ij = sum_k (Ah+Al)_ik (Bh+Bl)_kj for a list of
 * (i, j) pairs (row-major A and B). */
void oracle_exact_gemm_entries(int64_t K, const float *Ah, const float *Al,
                               int64_t lda, const float *Bh, const float *Bl,
                               int64_t ldb, const int64_t *rows,
                               const int64_t *cols, int64_t count,
                               int64_t *limbs_out)
{
    for (int64_t t = 0; t < count; ++t) {
        int64_t i = rows[t], j = cols[t];
        oracle_exact_dot_ff(Ah + i * lda, Al + i * lda, 1, Bh + j, Bl + j, ldb,
                            K, limbs_out + t * LA_LIMBS);
    }
}

/* acc += sign * v for one binary32 value. */
static void la_add_f32(long_acc *acc, float v, int sign)
{
    int64_t m;
    int e;
    f32_decompose(v, &m, &e);
    la_add_scaled(acc, sign * m, e);
}

/* The accumulated value rounded to binary64 (for reporting errors only).
 * The magnitude is summed limb by limb from the top, after the sign has been
 * taken out, so that no cancellation occurs in the conversion. */
static double la_to_double(long_acc *acc)
{
    la_normalise(acc);
    int neg = acc->limb[LA_LIMBS - 1] < 0;
    if (neg) {
        for (int k = 0; k < LA_LIMBS; ++k)
            acc->limb[k] = -acc->limb[k];
        la_normalise(acc);
    }
    double v = 0.0;
    for (int k = LA_LIMBS - 1; k >= 0; --k)
        v += ldexp((double)acc->limb[k], 32 * k + LA_EMIN);
    return neg ? -v : v;
}

/* Errors of operator results against the exact values: the measurement
 * behind an accuracy table of the shape of Table 5 (section 6.1).  For each
 * i, with E the exact result of the operation on the inputs:
 *   op 0 Add22: E = ah + al + bh + bl, bound = max(2^-24 |al + bl|,
 *               2^-44 |E|) (Add22 theorem)
 *   op 1 Mul22: E = (ah + al)(bh + bl), bound = 2^-44 |E| (Mul22 theorem)
 *   op 2 Add12: E = ah + bh (al, bl unused), bound = 0 (Add12 theorem: exact)
 *   op 3 Mul12: E = ah * bh (al, bl unused), bound = 0 (Mul12 theorem: exact)
 *   op 4 Div22: quotient q = rh + rl of a / b, bound 2^-44 relative
 *   op 5 FMA-based product (DWTimesDW3): as op 1, bound 5u^2 |E|
 *   op 6 reciprocal-based division (DWDivDW3): as op 4, bound 9.8u^2
 * For ops 0-3 and 5 the error err = (rh + rl) - E is formed without
 * rounding.  For the divisions, E = ah + al (the dividend) and
 * err = q (bh + bl) - E, also exact: |err| / |E| = |q - a/b| / |a/b| is the
 * quotient's relative error.  Then
 *   rel[i]   = |err| / |E|    (0 if err = 0; +inf if E = 0 != err)
 *   ratio[i] = |err| / bound  (0 if err = 0; +inf if bound = 0 != err)
 * rounded to binary64.  Returns -1 for an unknown op. */
int oracle_ff_errors(int op, const float *ah, const float *al, const float *bh,
                     const float *bl, const float *rh, const float *rl,
                     int64_t n, double *rel, double *ratio)
{
    if (op < 0 || op > 6)
        return -1;
    const int is_div = (op == 4 || op == 6);
    for (int64_t i = 0; i < n; ++i) {
        long_acc exact, lo;
        memset(&exact, 0, sizeof(exact));
        memset(&lo, 0, sizeof(lo));
        switch (op) {
        case 0:
            la_add_f32(&exact, ah[i], 1);
            la_add_f32(&exact, al[i], 1);
            la_add_f32(&exact, bh[i], 1);
            la_add_f32(&exact, bl[i], 1);
            la_add_f32(&lo, al[i], 1);
            la_add_f32(&lo, bl[i], 1);
            break;
        case 1:
        case 5:
            la_add_product(&exact, ah[i], bh[i]);
            la_add_product(&exact, ah[i], bl[i]);
            la_add_product(&exact, al[i], bh[i]);
            la_add_product(&exact, al[i], bl[i]);
            break;
        case 2:
            la_add_f32(&exact, ah[i], 1);
            la_add_f32(&exact, bh[i], 1);
            break;
        case 3:
            la_add_product(&exact, ah[i], bh[i]);
            break;
        default:
            la_add_f32(&exact, ah[i], 1);
            la_add_f32(&exact, al[i], 1);
            break;
        }
        long_acc err = exact;
        for (int k = 0; k < LA_LIMBS; ++k)
            err.limb[k] = -err.limb[k];
        if (is_div) {
            la_add_product(&err, rh[i], bh[i]);
            la_add_product(&err, rh[i], bl[i]);
            la_add_product(&err, rl[i], bh[i]);
            la_add_product(&err, rl[i], bl[i]);
        } else {
            la_add_f32(&err, rh[i], 1);
            la_add_f32(&err, rl[i], 1);
        }
        double e = fabs(la_to_double(&err));
        double big = fabs(la_to_double(&exact));
        double bound = 0.0;
        if (op == 0) {
            double lo_mag = fabs(la_to_double(&lo));
            double b1 = ldexp(lo_mag, -24), b2 = ldexp(big, -44);
            bound = b1 > b2 ? b1 : b2;
        } else if (op == 1 || op == 4) {
            bound = ldexp(big, -44);
        } else if (op == 5) {
            bound = 5.0 * ldexp(big, -48);
        } else if (op == 6) {
            bound = 9.8 * ldexp(big, -48);
        }
        rel[i] = e == 0.0 ? 0.0 : (big == 0.0 ? INFINITY : e / big);
        ratio[i] = e == 0.0 ? 0.0 : (bound == 0.0 ? INFINITY : e / bound);
    }
    return 0;
}

/* Exact |A| |B| entries: sum_k |(Ah+Al)_ik| |(Bh+Bl)_kj|, the normwise scale
 * for GEMM errors.  |Ah + Al| is taken with the sign of Ah + Al, which for a
 * float-float number is the sign of Ah (or of Al when Ah is zero). */
void oracle_exact_absgemm_entries(int64_t K, const float *Ah, const float *Al,
                                  int64_t lda, const float *Bh, const float *Bl,
                                  int64_t ldb, const int64_t *rows,
                                  const int64_t *cols, int64_t count,
                                  int64_t *limbs_out)
{
    for (int64_t t = 0; t < count; ++t) {
        int64_t i = rows[t], j = cols[t];
        long_acc acc;
        memset(&acc, 0, sizeof(acc));
        for (int64_t k = 0; k < K; ++k) {
            float a = Ah[i * lda + k], al = Al[i * lda + k];
            float b = Bh[k * ldb + j], bl = Bl[k * ldb + j];
            float sa = (a > 0.0f || (a == 0.0f && al > 0.0f)) ? 1.0f : -1.0f;
            float sb = (b > 0.0f || (b == 0.0f && bl > 0.0f)) ? 1.0f : -1.0f;
            a *= sa; al *= sa; b *= sb; bl *= sb;
            la_add_product(&acc, a, b);
            la_add_product(&acc, a, bl);
            la_add_product(&acc, al, b);
            la_add_product(&acc, al, bl);
        }
        la_store(&acc, limbs_out + t * LA_LIMBS);
    }
}
