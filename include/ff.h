/*
 * ff.h -- C ABI of libff: float-float arithmetic on AMD Instinct MI355X (gfx950).
 *
 * A float-float number is the unevaluated sum hi + lo of two IEEE binary32
 * words (Da Graca & Defour, "Implementation of float-float operators on
 * graphics hardware", section 4: the double-double format carried over to
 * single precision).  Arrays of float-float numbers are stored as two
 * separate planes (structure of arrays): hi[0..n) and lo[0..n).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Memory    Every array pointer is a DEVICE pointer owned by the caller (for
 *           example memory allocated by PyTorch on the current device).  The
 *           library never allocates, frees or retains device memory; scratch
 *           space, where needed, is a caller-provided workspace whose size is
 *           returned by the matching *_workspace_size() function.  The one
 *           exception is ff_dot_batched_noalloc, whose scratch is a static
 *           device array of the library (see there).
 * Streams   `stream` is a hipStream_t passed as void*; NULL is the null
 *           stream.  Work is enqueued asynchronously on that stream, on the
 *           current HIP device, and is complete when the stream is.
 * Checks    Arguments are validated on the host, synchronously, before any
 *           HIP call: an invalid call returns an error status and enqueues
 *           nothing.  A size of zero is a valid no-op returning FF_OK.
 *           Floating-point data never cause an error: NaN and infinity
 *           propagate as IEEE arithmetic makes them, and division by zero
 *           gives IEEE infinities/NaN (not a meaningful float-float value).
 * Alignment Float pointers must be 4-byte aligned (FF_ERR_ALIGN otherwise).
 *           Where an entry point has a float4 path for 16-byte aligned
 *           planes, its comment says when that path runs.
 * Aliasing  Elementwise entry points (the float-float operators, ff_copy,
 *           the paper's stream operators, the polynomial evaluators) allow
 *           an output plane to be the same array as an input plane (in
 *           place); partially overlapping arrays are undefined.  The outputs
 *           of the reductions, products, matrix-vector products, backward
 *           passes and conversions must not overlap any input.
 * Numerics  Device code is compiled with contraction off, binary32 denormals
 *           preserved and correctly rounded binary32 division, so that each
 *           operator performs exactly the operation sequence documented for
 *           it; elementwise results are therefore reproducible bit for bit.
 * Threads   Entry points hold no mutable global state (apart from the
 *           per-device address of ff_dot_batched_noalloc's scratch) and may
 *           be called from several host threads.
 * Graphs    Every entry point except ff_dot_batched_autotune only enqueues
 *           kernels: no allocation, no memset, no host wait.  A sequence of
 *           calls can therefore be captured into a HIP graph and replayed;
 *           workspaces and outputs are then bound at capture time.
 */
#ifndef FF_H
#define FF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FF_ABI_VERSION 1

typedef int32_t ff_status;

#define FF_OK              0 /* success (work enqueued, or nothing to do)   */
#define FF_ERR_NULL        1 /* a required pointer is NULL                  */
#define FF_ERR_SIZE        2 /* negative or inconsistent size / dimension   */
#define FF_ERR_ALIGN       3 /* pointer not aligned to its element type     */
#define FF_ERR_WORKSPACE   4 /* workspace missing or smaller than required  */
#define FF_ERR_UNSUPPORTED 5 /* the launch found no gfx950 code for the     */
                             /* current device                              */
#define FF_ERR_HIP         6 /* the HIP runtime reported an error (launch)  */
#define FF_ERR_ARG         7 /* invalid enumeration value or option         */

/* Human-readable name of a status code (static string, never NULL). */
const char *ff_status_str(ff_status status);

/* FF_ABI_VERSION of the built library. */
int32_t ff_abi_version(void);

/* Static string describing how the library was built: target, contraction,
 * denormal mode, division mode, TwoProd variants. */
const char *ff_build_info(void);

/* Text of the last HIP error seen by an entry point on the calling host
 * thread ("" if none). */
const char *ff_last_error(void);

/* ------------------------------------------------------------------------ */
/* Elementwise operators on n float-float pairs:                            */
/*     (r_hi[i], r_lo[i]) = OP((a_hi[i], a_lo[i]), (b_hi[i], b_lo[i]))      */
/* All six planes (four in, two out) hold n binary32 values.  Results are  */
/* bit-identical to the documented binary32 operation sequence, whatever   */
/* the alignment and launch form (float4 groups below 2^22 elements when   */
/* every plane is 16-byte aligned, 4-byte accesses otherwise).  Errors:    */
/* FF_ERR_SIZE (n < 0), FF_ERR_NULL (a NULL plane, n > 0), FF_ERR_ALIGN,   */
/* FF_ERR_HIP.                                                              */
/* ------------------------------------------------------------------------ */

/* Add22 (section 4.1, Add22 theorem): r = ah (+) bh; if |ah| >= |bh| then
 * s = (((ah (-) r) (+) bh) (+) bl) (+) al, else s = (((bh (-) r) (+) ah)
 * (+) al) (+) bl; result Add12(r, s), with the branch-free six-operation
 * Add12 (Add12 theorem).  |error| <= max(2^-24 |al + bl|, 2^-44 |a + b|). */
ff_status ff_add(const float *a_hi, const float *a_lo, const float *b_hi,
                 const float *b_lo, float *r_hi, float *r_lo, int64_t n,
                 void *stream);

/* Sub22: Add22 of a and -b (negating both words of b is exact). */
ff_status ff_sub(const float *a_hi, const float *a_lo, const float *b_hi,
                 const float *b_lo, float *r_hi, float *r_lo, int64_t n,
                 void *stream);

/* Mul22 (section 4.1, Mul22 theorem) with the exact product of the high
 * words from one fused multiply-add, (t1, t2) = (ah*bh, fma(ah, bh, -t1));
 * t3 = ((ah (x) bl) (+) (al (x) bh)) (+) t2; result Add12(t1, t3).
 * (The paper prints Add12(t1, t2) as the last step, which leaves t3 unused;
 * Add12(t1, t3) is the operator its theorem describes.)
 * Relative error <= 2^-44. */
ff_status ff_mul(const float *a_hi, const float *a_lo, const float *b_hi,
                 const float *b_lo, float *r_hi, float *r_lo, int64_t n,
                 void *stream);

/* Mul22 with the high-word product computed by Dekker's Mul12 through Split
 * with the constant 2^12 + 1 (section 4.1, Split and Mul12 theorems), as the
 * paper does on hardware without a fused multiply-add.  Bit-identical to
 * ff_mul whenever the product's error word is representable (no underflow). */
ff_status ff_mul_dekker(const float *a_hi, const float *a_lo,
                        const float *b_hi, const float *b_lo, float *r_hi,
                        float *r_lo, int64_t n, void *stream);

/* Div22 (not defined by the paper; Dekker's div2, the source the paper cites
 * for Split and Mul12): c = ah (/) bh; (u, uu) = c*bh exactly (FMA);
 * cc = ((((ah (-) u) (-) uu) (+) al) (-) (c (x) bl)) (/) bh;
 * result Add12(c, cc).  (/) is correctly rounded binary32 division.
 * Relative error <= 2^-44 is the tested bar; no proof is claimed (the worst
 * measured on 2^24 random pairs of either workload is 2^-45.0). */
ff_status ff_div(const float *a_hi, const float *a_lo, const float *b_hi,
                 const float *b_lo, float *r_hi, float *r_lo, int64_t n,
                 void *stream);

/* Cancellation-safe float-float addition and subtraction (not in the
 * paper): r = a + b (resp. a - b) by the AccurateDWPlusDW algorithm of
 * Joldes, Muller and Popescu (ACM TOMS 2017):
 *   (sh, sl) = Add12(a_hi, b_hi); (th, tl) = Add12(a_lo, b_lo);
 *   c = sl (+) th; (vh, vl) = Fast2Sum(sh, c); w = tl (+) vl;
 *   (r_hi, r_lo) = Fast2Sum(vh, w).
 * Its error is relative in every case, |r - (a + b)| <= 3u^2/(1 - 4u)
 * |a + b| with u = 2^-24, where the paper's Add22 bound (section 4.1,
 * Add22 theorem) is not relative once the operands cancel; it costs about
 * twice Add22's operations, which stay far below the HBM bound.
 * Arguments, layout and errors as for ff_add. */
ff_status ff_add_accurate(const float *a_hi, const float *a_lo,
                          const float *b_hi, const float *b_lo, float *r_hi,
                          float *r_lo, int64_t n, void *stream);
ff_status ff_sub_accurate(const float *a_hi, const float *a_lo,
                          const float *b_hi, const float *b_lo, float *r_hi,
                          float *r_lo, int64_t n, void *stream);

/* FMA-based float-float product (not in the paper): r = a * b by the
 * DWTimesDW3 algorithm of Joldes, Muller and Popescu (ACM TOMS 2017):
 *   (ch, cl1) = TwoProd(a_hi, b_hi) (FMA); tl0 = a_lo (x) b_lo;
 *   tl1 = fma(a_hi, b_lo, tl0); cl2 = fma(a_lo, b_hi, tl1);
 *   cl3 = cl1 (+) cl2; (r_hi, r_lo) = Fast2Sum(ch, cl3).
 * Relative error <= 5u^2 (u = 2^-24), against 2^-44 = 16u^2 for the paper's
 * Mul22 (section 4.1, Mul22 theorem), in fewer operations.
 * Arguments, layout and errors as for ff_add. */
ff_status ff_mul_accurate(const float *a_hi, const float *a_lo,
                          const float *b_hi, const float *b_lo, float *r_hi,
                          float *r_lo, int64_t n, void *stream);

/* Reciprocal-based float-float division (not in the paper): r = a / b by the
 * DWDivDW3 algorithm of Joldes, Muller and Popescu (ACM TOMS 2017):
 *   th = 1 (/) b_hi; e = (fma(-b_hi, th, 1), -b_lo (x) th) joined by Add12;
 *   m = e * th + th (float-float times float, then plus float, each ending in
 *   Fast2Sum); r = a * m by ff_mul_accurate's sequence.
 * Relative error <= 9.8u^2.  One correctly rounded division per element
 * (ff_div has two).  Valid for 2^-126 < |b_hi| < 2^126, where 1/b_hi is a
 * normal number; outside, as for b = 0, the result is not a float-float
 * quotient (no error is raised).
 * Arguments, layout and errors as for ff_add. */
ff_status ff_div_accurate(const float *a_hi, const float *a_lo,
                          const float *b_hi, const float *b_lo, float *r_hi,
                          float *r_lo, int64_t n, void *stream);

/* ------------------------------------------------------------------------ */
/* Batched float-float dot products (reductions)                            */
/* ------------------------------------------------------------------------ */
/*
 * nvec independent dot products over concatenated vectors: vector v owns the
 * elements [offsets[v], offsets[v+1]) of x and y.  Every term is formed
 * exactly -- TwoProd(x_i, y_i) for binary32 inputs, Mul22 for float-float
 * inputs -- and accumulated with Add22 (section 4.1) in float-float.  The
 * paper defines no reduction; compensated summation is its stated future
 * work (section 7).
 *
 * Execution: four launches on `stream`: a planning launch (chunk counts and
 * their scan), one writing each chunk's element range, one reducing the
 * chunks -- one workgroup per chunk of block * unroll elements, launched in
 * chunk order so that the resident workgroups stream memory together; each
 * thread adds its `unroll` terms in order into a float-float accumulator,
 * then a butterfly of Add22 over lane shuffles and the wavefronts' sums in
 * index order give the chunk's float-float partial -- and one combining
 * each vector's partials (one wavefront per vector, an Add22 tree of fixed
 * shape).  No atomics are used: for a given cfg the result is bitwise
 * reproducible run to run.  Different cfg values may give different
 * (equally valid) last bits.  Any 4-byte alignment of the inputs.
 *
 * Accuracy: |result - exact| is bounded by (tree depth) * 2^-44 * sum|x_i y_i|
 * in the worst case; on random data it is far smaller (2^-47.1 sum|x_i y_i|
 * at worst over a batch of 4096 vectors of 64 to 2^20 normal(0,1) terms).
 */

/* Launch shape of the batched reductions.  Zero fields select the entry
 * point's default: 256 threads by 32 elements per thread (chunks of 8192
 * elements) for every input kind. */
typedef struct ff_dot_cfg {
    int32_t block;  /* threads per workgroup: 64, 128, 256 or 512            */
    int32_t chunk;  /* elements per chunk: 0 or block * unroll (with unroll
                       0, a chunk given sets unroll = chunk / block)         */
    int32_t grid;   /* reserved: must be 0 (one workgroup per chunk)         */
    int32_t unroll; /* elements per thread and input plane: 1, 2, 4, 8, 16
                       or 32                                                 */
} ff_dot_cfg;

/* Bytes of device workspace the batched reductions need for nvec vectors
 * holding total_len elements in all, with this cfg (zero fields resolved
 * with the default chunk, 8192, which every entry point shares).  Returns 0
 * for invalid arguments. */
size_t ff_dot_batched_workspace_size(int64_t total_len, int32_t nvec,
                                     const ff_dot_cfg *cfg);

/* out[v] = sum over [offsets[v], offsets[v+1]) of x_i * y_i, binary32
 * inputs, float-float result (out_hi[v], out_lo[v]).
 *   x, y       device, total_len binary32 each
 *   offsets    device, nvec + 1 int64, non-decreasing, offsets[0] >= 0,
 *              offsets[nvec] <= total_len (violations give unspecified
 *              results but never access memory outside the arrays)
 *   cfg        host pointer or NULL (defaults)
 *   ws         device workspace of ws_bytes >= the size queried above;
 *              it must not be shared by launches that may overlap
 *   out_hi/lo  device, nvec binary32 each; an empty vector gives (0, 0)
 * Errors: FF_ERR_SIZE (nvec < 0, total_len < 0), FF_ERR_NULL, FF_ERR_ALIGN,
 * FF_ERR_ARG (invalid cfg), FF_ERR_WORKSPACE, FF_ERR_HIP. */
ff_status ff_dot_batched(const float *x, const float *y,
                         const int64_t *offsets, int32_t nvec,
                         int64_t total_len, const ff_dot_cfg *cfg, void *ws,
                         size_t ws_bytes, float *out_hi, float *out_lo,
                         void *stream);

/* As ff_dot_batched for float-float inputs: the terms are Mul22 products
 * (FMA TwoProd) of (x_hi, x_lo) and (y_hi, y_lo). */
ff_status ff_dot_ff_batched(const float *x_hi, const float *x_lo,
                            const float *y_hi, const float *y_lo,
                            const int64_t *offsets, int32_t nvec,
                            int64_t total_len, const ff_dot_cfg *cfg, void *ws,
                            size_t ws_bytes, float *out_hi, float *out_lo,
                            void *stream);

/* Batched float-float sums: out[v] = sum over [offsets[v], offsets[v+1]) of
 * x_i (binary32 terms (x_i, 0)), accumulated with Add22 exactly as the
 * dots.  Arguments and errors as for ff_dot_batched. */
ff_status ff_sum_batched(const float *x, const int64_t *offsets, int32_t nvec,
                         int64_t total_len, const ff_dot_cfg *cfg, void *ws,
                         size_t ws_bytes, float *out_hi, float *out_lo,
                         void *stream);

/* As ff_sum_batched for float-float terms (x_hi[i], x_lo[i]). */
ff_status ff_sum_ff_batched(const float *x_hi, const float *x_lo,
                            const int64_t *offsets, int32_t nvec,
                            int64_t total_len, const ff_dot_cfg *cfg, void *ws,
                            size_t ws_bytes, float *out_hi, float *out_lo,
                            void *stream);

/* Compensated batched dot products and sums (the paper's named future work,
 * section 7): Dot2 and Sum2 of Ogita, Rump and Oishi (SIAM J. Sci. Comput.
 * 2005) on binary32 inputs.  Each vector keeps a running binary32 sum p and
 * adds the exact rounding error of every step (TwoSum) and every product
 * (TwoProduct, FMA form) into a second binary32 word s; chunk partials
 * (p, s) merge as (p, q) = TwoSum(p1, p2), s = (s1 + s2) + q.  The result
 * is returned as Add12(p, s): out_hi[v] is the algorithm's binary32 result
 * p (+) s, out_lo[v] the remainder.  Error: |out_hi - x.y| <= u |x.y| +
 * gamma_n^2 sum |x_i y_i| (u = 2^-24, gamma_n = n u / (1 - n u)), the
 * accuracy of the working precision squared; fewer operations per term than
 * float-float accumulation (no renormalisation per step).  Same execution,
 * workspace, launch shape, arguments and errors as ff_dot_batched /
 * ff_sum_batched (ff_dot_batched_workspace_size applies). */
ff_status ff_dot2_batched(const float *x, const float *y,
                          const int64_t *offsets, int32_t nvec,
                          int64_t total_len, const ff_dot_cfg *cfg, void *ws,
                          size_t ws_bytes, float *out_hi, float *out_lo,
                          void *stream);
ff_status ff_sum2_batched(const float *x, const int64_t *offsets, int32_t nvec,
                          int64_t total_len, const ff_dot_cfg *cfg, void *ws,
                          size_t ws_bytes, float *out_hi, float *out_lo,
                          void *stream);

/* Capacity of the static scratch array of ff_dot_batched_noalloc (bytes). */
#define FF_NOALLOC_SCRATCH_BYTES ((size_t)16 << 20)

/* ff_dot_batched without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same kernels, results (bit for bit for
 * the same cfg), arguments and errors as ff_dot_batched; its scratch is a
 * static device array of FF_NOALLOC_SCRATCH_BYTES inside the library, one
 * copy per device, held until the process ends (its device address is looked
 * up once per device on the first call there).  No allocation of any kind.
 * Limit: the batch's workspace (ff_dot_batched_workspace_size(total_len,
 * nvec, cfg), here resolved with ff_dot_batched's own defaults) must not
 * exceed FF_NOALLOC_SCRATCH_BYTES, otherwise FF_ERR_WORKSPACE (with the
 * default cfg, for example, 4096 vectors of up to 5.6e9 elements in all).
 * Nothing in the scratch needs to start at zero: every word a launch reads
 * was written earlier in the same call.  Every call on one device
 * shares that device's array, so calls that may overlap on one device (two
 * streams, two host threads) race and give unspecified results; calls on
 * one stream are ordered and safe.  Errors: those of ff_dot_batched, and
 * FF_ERR_UNSUPPORTED for a device index of 64 or more. */
ff_status ff_dot_batched_noalloc(const float *x, const float *y,
                                 const int64_t *offsets, int32_t nvec,
                                 int64_t total_len, const ff_dot_cfg *cfg,
                                 float *out_hi, float *out_lo, void *stream);

/* Launch-shape autotuner for ff_dot_batched on this batch: times every
 * candidate (block 64/128/256/512 x unroll 4/8/16/32) whose workspace fits
 * in ws_bytes, `reps` launches each after one untimed launch, with HIP
 * events on `stream`, and returns the fastest in *best with its mean time in
 * *best_ms.  SYNCHRONOUS: waits for each candidate.  out_hi/out_lo receive
 * the last candidate's result.  Errors: those of ff_dot_batched, FF_ERR_NULL
 * (best/best_ms), FF_ERR_ARG (reps < 1), FF_ERR_WORKSPACE (no candidate
 * fits). */
ff_status ff_dot_batched_autotune(const float *x, const float *y,
                                  const int64_t *offsets, int32_t nvec,
                                  int64_t total_len, void *ws, size_t ws_bytes,
                                  float *out_hi, float *out_lo, int32_t reps,
                                  void *stream, ff_dot_cfg *best,
                                  float *best_ms);

/* ------------------------------------------------------------------------ */
/* Matrix-vector product and its backward pass (differentiation)            */
/* ------------------------------------------------------------------------ */
/*
 * A is an M x N float-float matrix, row-major, two planes with leading
 * dimension lda >= N (elements); vectors are float-float planes.  Every term
 * is a Mul22 product (FMA TwoProd) and sums use Add22 (section 4.1).
 *
 * algo FF_MATVEC_FAST  -- tiled kernels: one workgroup per pair of rows
 *                         sharing each load of x (forward);
 *                         one fused pass over A writing dA and per-band
 *                         partial column sums of A^T g (backward), combined
 *                         in band order by a second small launch.
 * algo FF_MATVEC_PLAIN -- the plain float-float loops: one thread per row
 *                         (forward) or per column (backward), sums in index
 *                         order, a separate launch for dA.  Bit-identical to
 *                         the sequential definition.
 */
#define FF_MATVEC_FAST  0
#define FF_MATVEC_PLAIN 1

/* y = A x.  y_hi/y_lo: M values each.  Errors: FF_ERR_SIZE (M, N < 0 or
 * lda < N), FF_ERR_NULL, FF_ERR_ALIGN, FF_ERR_ARG (algo), FF_ERR_HIP. */
ff_status ff_matvec(int64_t M, int64_t N, const float *A_hi, const float *A_lo,
                    int64_t lda, const float *x_hi, const float *x_lo,
                    float *y_hi, float *y_lo, int32_t algo, void *stream);

/* Workspace bytes of ff_matvec_backward (partial column sums of the fast
 * algorithm; 0 for the plain one). */
size_t ff_matvec_backward_workspace_size(int64_t M, int64_t N, int32_t algo);

/* Backward pass of y = A x for an upstream gradient g = dL/dy (M values):
 *   dA = g x^T      dA_ij = Mul22(g_i, x_j), bit-identical to Mul22
 *   dx = A^T g      dx_j  = sum_i Mul22(g_i, A_ij) with Add22
 * dA (leading dimension ldda >= N) may be NULL to skip it; dx may be NULL to
 * skip it.  The fast algorithm reads A once and writes dA once in the same
 * pass.  Errors as ff_matvec, plus FF_ERR_WORKSPACE. */
ff_status ff_matvec_backward(int64_t M, int64_t N, const float *A_hi,
                             const float *A_lo, int64_t lda, const float *x_hi,
                             const float *x_lo, const float *g_hi,
                             const float *g_lo, float *dA_hi, float *dA_lo,
                             int64_t ldda, float *dx_hi, float *dx_lo,
                             int32_t algo, void *ws, size_t ws_bytes,
                             void *stream);

/* Backward pass of the float-float dot s = sum_i x_i y_i for an upstream
 * gradient g = dL/ds (ONE float-float value, device pointers g_hi, g_lo):
 *   dx_i = Mul22(g, y_i),  dy_i = Mul22(g, x_i)   (elementwise, n values).
 * Either output pair may be NULL to skip it. */
ff_status ff_dot_backward(const float *g_hi, const float *g_lo,
                          const float *x_hi, const float *x_lo,
                          const float *y_hi, const float *y_lo, float *dx_hi,
                          float *dx_lo, float *dy_hi, float *dy_lo, int64_t n,
                          void *stream);

/* Backward pass of the batched float-float dot (ff_dot_batched /
 * ff_dot_ff_batched) for per-vector upstream gradients g_v (device, nvec
 * float-float values g_hi[v] + g_lo[v]): every element i of vector v, i in
 * [offsets[v], offsets[v+1]), gets
 *   dx_i = Mul22(g_v, y_i),  dy_i = Mul22(g_v, x_i)   (FMA TwoProd),
 * and every element of no vector (before offsets[0], from offsets[nvec] on)
 * gets zero gradients, so all total_len entries of each output are written.
 * x_lo / y_lo may be NULL (binary32 inputs, zero low words).  Either output
 * pair may be NULL to skip it; x is read only for dy, y only for dx.
 * offsets: device, nvec + 1 int64, non-decreasing within [0, total_len],
 * as for the forward (violations give unspecified gradients, never accesses
 * outside the arrays: offsets are clamped to [0, total_len]).
 * ws: device workspace of at least
 * ff_dot_batched_backward_workspace_size(total_len) bytes, 16-byte aligned,
 * caller-owned; it holds, per block of 256 elements, the vector owning the
 * block's first element with its gradient (written by a first launch, read
 * by the second), so it must not be shared by calls that may overlap.
 * Errors: FF_ERR_SIZE (nvec < 0, total_len < 0, or total_len beyond
 * (2^31 - 1) * 256), FF_ERR_NULL, FF_ERR_ALIGN
 * (offsets not 8-byte, a plane not 4-byte or ws not 16-byte aligned),
 * FF_ERR_WORKSPACE (ws NULL or too small), FF_ERR_HIP.
 * total_len = 0, or no output wanted, is a no-op (ws is not read). */
size_t ff_dot_batched_backward_workspace_size(int64_t total_len);
ff_status ff_dot_batched_backward(const float *g_hi, const float *g_lo,
                                  const int64_t *offsets, int32_t nvec,
                                  int64_t total_len, const float *x_hi,
                                  const float *x_lo, const float *y_hi,
                                  const float *y_lo, float *dx_hi,
                                  float *dx_lo, float *dy_hi, float *dy_lo,
                                  void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------ */
/* Matrix product C = A B                                                   */
/* ------------------------------------------------------------------------ */
/*
 * A (M x K), B (K x N), C (M x N): float-float, row-major, two planes each
 * with leading dimensions lda >= K, ldb >= N, ldc >= N.  C is overwritten.
 * The paper defines no matrix product; both algorithms build on its
 * operators and error-free transformations.
 *
 * FF_GEMM_FMA_LOOP    the plain float-float GEMM: C_ij = Add22
 *                     accumulation, k ascending, of Mul22(A_ik, B_kj)
 *                     (section 4.1).  Bit-identical to that definition.
 * FF_GEMM_SLICED_I8   matrix-core path: each row of A and column of B is
 *                     scaled by a power of two and cut into 7 signed 8-bit
 *                     digits; the 28 digit-pair products that carry weight
 *                     above 2^-56 of the row/column scales run as exact
 *                     integer GEMMs (int8 inputs, int32 accumulation) and
 *                     are recombined exactly; one final rounding to
 *                     float-float.  No binary64 arithmetic.
 * FF_GEMM_SLICED_BF16 as above with the digits held in BF16 (exact for
 *                     |d| <= 128) and FP32 matrix-core accumulation, whose
 *                     partial sums are moved to integer accumulators before
 *                     they can exceed 2^24 (so they stay exact).
 * Sliced accuracy: |C_ij - exact| <= 2^-44 * (|A| |B|)_ij when the rows of
 * A and columns of B do not span extreme dynamic ranges (normal(0,1) data at
 * 4096^3: 2^-51.6 at worst).  In general, with 2^e_i the power of two above
 * row i's largest |A_ik| and 2^f_j the one above column j's largest |B_kj|:
 *   |C_ij - exact| <= 2^(e_i - 54) sum_k |B_kj|
 *                   + 2^(f_j - 54) sum_k (|A_ik| + 2^(e_i - 54))
 *                   + K 2^(e_i + f_j - 47) + 2^-47 |C_ij|
 * (digit rounding, dropped digit pairs, final rounding).  Rows and columns
 * spanning 40 binades measured 2^-11.3 normwise, inside this bound; the FMA
 * loop has no such limit.
 * Inputs must be finite float-float numbers with |lo| <= ulp(hi).
 * Workspace: 0 bytes for the FMA loop; digit planes (7 (M+N) K bytes for
 * int8, twice that for BF16, rounded up to 64-row / 64-byte tiles) plus
 * scales for the sliced paths.
 * Errors: FF_ERR_SIZE, FF_ERR_NULL, FF_ERR_ALIGN, FF_ERR_ARG (algo),
 * FF_ERR_WORKSPACE, FF_ERR_HIP.
 */
#define FF_GEMM_FMA_LOOP    0
#define FF_GEMM_SLICED_BF16 1
#define FF_GEMM_SLICED_I8   2

/* Workspace bytes ff_gemm needs for this shape and algorithm (0 for an
 * invalid request or the FMA loop). */
size_t ff_gemm_workspace_size(int64_t M, int64_t N, int64_t K, int32_t algo);

ff_status ff_gemm(int64_t M, int64_t N, int64_t K, const float *A_hi,
                  const float *A_lo, int64_t lda, const float *B_hi,
                  const float *B_lo, int64_t ldb, float *C_hi, float *C_lo,
                  int64_t ldc, int32_t algo, void *ws, size_t ws_bytes,
                  void *stream);

/* ------------------------------------------------------------------------ */
/* Error-free transforms and binary32 reference operators                   */
/* ------------------------------------------------------------------------ */
/*
 * The building blocks the paper times beside its float-float operators
 * (section 6, Tables 3 and 4), as stream operators over n binary32 elements
 * with the same load/store pattern as the float-float operators:
 *   ff_add12         (s_i, r_i) = Add12(a_i, b_i): s = a (+) b and
 *                    r = (a + b) - s exactly (section 4.1, Add12 theorem;
 *                    the branch-free six-operation form)
 *   ff_mul12         (x_i, y_i): x = a (x) b, y = fma(a, b, -x), which is
 *                    a*b - x exactly unless the error word underflows
 *   ff_mul12_dekker  (x_i, y_i) = Mul12(a_i, b_i) through Split with the
 *                    constant 4097 (section 4.1, Split and Mul12 theorems)
 *   ff_f32_add       r_i = a_i (+) b_i           (the tables' "Add")
 *   ff_f32_mul       r_i = a_i (x) b_i           (the tables' "Mul")
 *   ff_f32_mad       r_i = fma(a_i, b_i, c_i), one rounding (the tables'
 *                    "Mad"; gfx950 has no unfused binary32 multiply-add)
 * All pointers: device, caller-owned, n binary32 words each; an output may
 * alias an input exactly (in place), partial overlap is undefined.  Below
 * 2^22 elements, when every pointer is 16-byte aligned, a float4 path runs;
 * otherwise 4-byte accesses, one lane-contiguous element per lane and
 * plane at a time.  Results do not depend on the path.
 * Errors: FF_ERR_SIZE (n < 0), FF_ERR_NULL, FF_ERR_ALIGN (a pointer not
 * 4-byte aligned), FF_ERR_HIP.  n = 0 is a no-op. */
ff_status ff_add12(const float *a, const float *b, float *s, float *r,
                   int64_t n, void *stream);
ff_status ff_mul12(const float *a, const float *b, float *x, float *y,
                   int64_t n, void *stream);
ff_status ff_mul12_dekker(const float *a, const float *b, float *x, float *y,
                          int64_t n, void *stream);
ff_status ff_f32_add(const float *a, const float *b, float *r, int64_t n,
                     void *stream);
ff_status ff_f32_mul(const float *a, const float *b, float *r, int64_t n,
                     void *stream);
ff_status ff_f32_mad(const float *a, const float *b, const float *c, float *r,
                     int64_t n, void *stream);

/* ------------------------------------------------------------------------ */
/* Polynomial evaluation at many points (compensated algorithms, the        */
/* paper's future work, section 7)                                           */
/* ------------------------------------------------------------------------ */
/*
 * p(x) = sum_{i=0..degree} coef[i] x^i, coefficients in ascending order
 * (device memory, degree + 1 words per plane), evaluated independently at
 * each of the n points x_k; result k goes to y_k.
 *
 *   ff_horner_f32   Horner's rule in binary32: s = c_n; s = (s (x) x) (+) c_i.
 *                   Error <= gamma_2n(u) sum |c_i| |x|^i, u = 2^-24,
 *                   gamma_k(v) = k v / (1 - k v).
 *   ff_horner_comp  compensated Horner (CompHorner of Graillat, Langlois and
 *                   Louvet, 2005): (p, pi) = TwoProd(s, x) (FMA);
 *                   (s, sigma) = Add12(p, c_i); r = (r (x) x) (+) (pi (+)
 *                   sigma), r starting at 0; y = s (+) r.  Error <= u |p(x)|
 *                   + gamma_2n(u)^2 sum |c_i| |x|^i: as accurate as Horner in
 *                   twice the working precision, then rounded.
 *   ff_horner_ff    float-float Horner: s = (coef_hi[n], coef_lo[n]);
 *                   s = Add22(Mul22(s, x), c_i) (section 4.1 operators, FMA
 *                   TwoProd); the result is the float-float (y_hi, y_lo).
 *                   Error <= gamma_2n(2^-44) sum |c_i| |x|^i.
 * The bounds assume no underflow or overflow.  Results are bit-for-bit
 * those of the operation sequences above (no contraction, IEEE binary32).
 *
 * Arguments: coef / coef_hi (non-null) and coef_lo (null: zero low words);
 * x / x_hi (non-null) and x_lo (null: binary32 points); y / y_hi, y_lo
 * (non-null).  All device pointers, caller-owned, 4-byte aligned; the float4
 * path runs when every point and result plane is 16-byte aligned.  A result
 * plane may alias a point plane exactly (in place); coefficients must not
 * alias a result.
 * Errors: FF_ERR_NULL, FF_ERR_SIZE (degree < 0 or n < 0), FF_ERR_ALIGN,
 * FF_ERR_HIP.  n = 0 is a no-op. */
ff_status ff_horner_f32(const float *coef, int32_t degree, const float *x,
                        float *y, int64_t n, void *stream);
ff_status ff_horner_comp(const float *coef, int32_t degree, const float *x,
                         float *y, int64_t n, void *stream);
ff_status ff_horner_ff(const float *coef_hi, const float *coef_lo,
                       int32_t degree, const float *x_hi, const float *x_lo,
                       float *y_hi, float *y_lo, int64_t n, void *stream);

/* ------------------------------------------------------------------------ */
/* Conversions between binary64 and float-float (not in the paper)          */
/* ------------------------------------------------------------------------ */
/*
 * ff_from_f64: hi_i = fl32(x_i), lo_i = fl32(x_i - hi_i) (the difference is
 *   exact in binary64), so hi + lo = x to within 2^-48 |x| for x in the
 *   binary32 normal range.  Outside it the same sequence gives pairs that are
 *   not float-float numbers: x = +-inf gives (x, NaN); a finite x that rounds
 *   past the binary32 maximum gives (+-inf, -+inf); NaN gives (NaN, NaN).
 * ff_to_f64: x_i = (double) hi_i + (double) lo_i, one binary64 rounding
 *   (exact whenever the pair's bits fit in 53).
 * Pointers: device, caller-owned; binary64 plane 8-byte aligned, binary32
 * planes 4-byte aligned.  No aliasing between the binary64 and binary32
 * planes.
 * Errors: FF_ERR_SIZE (n < 0), FF_ERR_NULL, FF_ERR_ALIGN, FF_ERR_HIP.
 * n = 0 is a no-op. */
ff_status ff_from_f64(const double *x, float *hi, float *lo, int64_t n,
                      void *stream);
ff_status ff_to_f64(const float *hi, const float *lo, double *x, int64_t n,
                    void *stream);

/* ------------------------------------------------------------------------ */
/* Measurement probe                                                        */
/* ------------------------------------------------------------------------ */

/* dst[i] = src[i] for i < n (binary32): the streaming reference for the
 * roofline and the HBM counter calibration.  512 threads by 4
 * lane-contiguous elements with non-temporal 4-byte loads and stores, any
 * 4-byte alignment: the fastest copy measured on MI355X.  Errors as for the
 * elementwise operators. */
ff_status ff_copy(const float *src, float *dst, int64_t n, void *stream);

#ifdef __cplusplus
} /* extern "C" */
#endif

#endif /* FF_H */
