// ff_matvec.hip -- float-float matrix-vector product y = A x, its backward
// pass (dA = g x^T, dx = A^T g) and the backward pass of the float-float dot.
//
// A is M x N, row-major, hi and lo planes with leading dimension lda.  The
// forward pass reads A once (8 bytes per element) and performs Mul22 + Add22
// (~26 VALU) per element; the fused backward reads A once and writes dA once
// (16 bytes per element) with Mul22 (dA) + Mul22 + Add22 (dx) (~38 VALU).
// Both are HBM-bound on gfx950 (ridge ~9.8 binary32 operations per byte).
//
// Fast forward: one workgroup per pair of rows; lane t takes float4 groups
// t, t + BLOCK, ... of both rows (coalesced 1 KiB per wavefront load), each
// load of x serving both, keeps four Add22 accumulators per row (one per
// float4 component), then a wavefront butterfly and an in-order LDS combine
// give y_i.  x is re-read from L2 by every pair of rows.
// Fast backward: the workgroup grid is (column tiles) x (row bands); a
// thread owns four adjacent columns, walks the rows of its band, writes
// dA_ij = Mul22(g_i, x_j) and accumulates Mul22(g_i, A_ij) per column; the
// per-band partial column sums go to the workspace and a second launch adds
// them in band order.
#include <type_traits>

#include "ff_device.h"
#include "ff_host.h"

namespace ffk {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kRowBlock = 256;
// Backward band kernel: 128 threads (four columns each) by 128-row bands
// measured fastest at 8192 x 8192 (175-176 us against 183-185 us for 256
// threads by 64 rows; taller bands also halve the partial-sum traffic).
constexpr int kColBlock = 128;
constexpr int64_t kBandRows = 128;

// Fast forward for kRowsPerGroup rows at a time: the rows share each load
// of x, and each lane issues the loads of kRowUnroll float4 groups (both
// rows' planes and x) before any arithmetic.
constexpr int kRowsPerGroup = 2;
constexpr int kRowUnroll = 2;

template <int BLOCK, bool VEC>
__global__ __launch_bounds__(BLOCK) void matvec_rows(int64_t M, int64_t N,
                                                     const float *__restrict__ Ah,
                                                     const float *__restrict__ Al, int64_t lda,
                                                     const float *__restrict__ xh,
                                                     const float *__restrict__ xl,
                                                     float *__restrict__ yh, float *__restrict__ yl)
{
    constexpr int kWaves = BLOCK / 64;
    constexpr int R = kRowsPerGroup, U = kRowUnroll;
    __shared__ float2 part[R][kWaves];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int64_t r0 = static_cast<int64_t>(blockIdx.x) * R; r0 < M;
         r0 += static_cast<int64_t>(gridDim.x) * R) {
        // rows r0 .. r0 + R - 1; a row beyond M repeats row r0 (not stored)
        const float *rh[R], *rl[R];
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int64_t r = (r0 + q < M) ? r0 + q : r0;
            rh[q] = Ah + r * lda;
            rl[q] = Al + r * lda;
        }
        float2 acc[R][4];
#pragma unroll
        for (int q = 0; q < R; ++q)
#pragma unroll
            for (int k = 0; k < 4; ++k)
                acc[q][k] = make_float2(0.0f, 0.0f);
        auto add_term = [&](int q, int k, float ah, float al, float bh, float bl) {
            float ph, pl;
            ffd::mul22<false>(ah, al, bh, bl, ph, pl);
            ffd::add22(acc[q][k].x, acc[q][k].y, ph, pl, acc[q][k].x, acc[q][k].y);
        };
        int64_t j_scalar = tid;
        if (VEC) {
            const int64_t ng = N >> 2;
            const f32x4 *xh4 = reinterpret_cast<const f32x4 *>(xh);
            const f32x4 *xl4 = reinterpret_cast<const f32x4 *>(xl);
            int64_t g = tid;
            for (; g + (U - 1) * BLOCK < ng; g += U * BLOCK) {
                f32x4 bh[U], bl[U], ah[R][U], al[R][U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    bh[u] = xh4[g + u * BLOCK];
                    bl[u] = xl4[g + u * BLOCK];
#pragma unroll
                    for (int q = 0; q < R; ++q) {
                        ah[q][u] = __builtin_nontemporal_load(
                            reinterpret_cast<const f32x4 *>(rh[q]) + g + u * BLOCK);
                        al[q][u] = __builtin_nontemporal_load(
                            reinterpret_cast<const f32x4 *>(rl[q]) + g + u * BLOCK);
                    }
                }
#pragma unroll
                for (int u = 0; u < U; ++u)
#pragma unroll
                    for (int q = 0; q < R; ++q)
#pragma unroll
                        for (int k = 0; k < 4; ++k)
                            add_term(q, k, ah[q][u][k], al[q][u][k], bh[u][k], bl[u][k]);
            }
            for (; g < ng; g += BLOCK) {
                const f32x4 bh = xh4[g], bl = xl4[g];
#pragma unroll
                for (int q = 0; q < R; ++q) {
                    const f32x4 ah = __builtin_nontemporal_load(
                        reinterpret_cast<const f32x4 *>(rh[q]) + g);
                    const f32x4 al = __builtin_nontemporal_load(
                        reinterpret_cast<const f32x4 *>(rl[q]) + g);
#pragma unroll
                    for (int k = 0; k < 4; ++k)
                        add_term(q, k, ah[k], al[k], bh[k], bl[k]);
                }
            }
            j_scalar = 4 * ng + tid;
        }
        for (int64_t j = j_scalar; j < N; j += BLOCK) {
#pragma unroll
            for (int q = 0; q < R; ++q)
                add_term(q, 0, rh[q][j], rl[q][j], xh[j], xl[j]);
        }
#pragma unroll
        for (int q = 0; q < R; ++q) {
            float h = acc[q][0].x, l = acc[q][0].y, h2 = acc[q][2].x, l2 = acc[q][2].y;
            ffd::add22(h, l, acc[q][1].x, acc[q][1].y, h, l);
            ffd::add22(h2, l2, acc[q][3].x, acc[q][3].y, h2, l2);
            ffd::add22(h, l, h2, l2, h, l);
            ffd::wave_allreduce_add22(h, l);
            if (lane == 0)
                part[q][wave] = make_float2(h, l);
        }
        __syncthreads();
        if (tid < R && r0 + tid < M) {
            float th = part[tid][0].x, tl = part[tid][0].y;
#pragma unroll
            for (int k = 1; k < kWaves; ++k)
                ffd::add22(th, tl, part[tid][k].x, part[tid][k].y, th, tl);
            yh[r0 + tid] = th;
            yl[r0 + tid] = tl;
        }
        __syncthreads();
    }
}

// Plain forward: one thread per row, terms added in column order.
__global__ __launch_bounds__(256) void matvec_plain(int64_t M, int64_t N,
                                                    const float *__restrict__ Ah,
                                                    const float *__restrict__ Al, int64_t lda,
                                                    const float *__restrict__ xh,
                                                    const float *__restrict__ xl,
                                                    float *__restrict__ yh, float *__restrict__ yl)
{
    const int64_t r = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (r >= M)
        return;
    float h = 0.0f, l = 0.0f;
    for (int64_t j = 0; j < N; ++j) {
        float ph, pl;
        ffd::mul22<false>(Ah[r * lda + j], Al[r * lda + j], xh[j], xl[j], ph, pl);
        ffd::add22(h, l, ph, pl, h, l);
    }
    yh[r] = h;
    yl[r] = l;
}

// Fused backward over one row band: thread owns COLS adjacent columns.
template <int BLOCK, int COLS, bool WANT_DA, bool WANT_DX>
__global__ __launch_bounds__(BLOCK) void matvec_bwd_band(
    int64_t M, int64_t N, const float *__restrict__ Ah, const float *__restrict__ Al, int64_t lda,
    const float *__restrict__ xh, const float *__restrict__ xl, const float *__restrict__ gh,
    const float *__restrict__ gl, float *__restrict__ dAh, float *__restrict__ dAl, int64_t ldda,
    float2 *__restrict__ part)
{
    const int64_t c0 = (static_cast<int64_t>(blockIdx.x) * BLOCK + threadIdx.x) * COLS;
    if (c0 >= N)
        return;
    const int64_t i0 = static_cast<int64_t>(blockIdx.y) * kBandRows;
    const int64_t i1 = (i0 + kBandRows < M) ? i0 + kBandRows : M;
    float x_h[COLS], x_l[COLS];
    float2 acc[COLS];
#pragma unroll
    for (int k = 0; k < COLS; ++k) {
        acc[k] = make_float2(0.0f, 0.0f);
        if (WANT_DA) {
            x_h[k] = xh[c0 + k];
            x_l[k] = xl[c0 + k];
        }
    }
    // rows in pairs: both rows' loads are issued before any arithmetic
    constexpr int kRowPair = 2;
    auto row = [&](int64_t i, const float (&a_h)[COLS], const float (&a_l)[COLS]) {
        const float g_h = gh[i], g_l = gl[i];
        if (WANT_DA) {
            float d_h[COLS], d_l[COLS];
#pragma unroll
            for (int k = 0; k < COLS; ++k)
                ffd::mul22<false>(g_h, g_l, x_h[k], x_l[k], d_h[k], d_l[k]);
            if constexpr (COLS == 4) {
                const f32x4 vh = {d_h[0], d_h[1], d_h[2], d_h[3]};
                const f32x4 vl = {d_l[0], d_l[1], d_l[2], d_l[3]};
                __builtin_nontemporal_store(vh, reinterpret_cast<f32x4 *>(dAh + i * ldda + c0));
                __builtin_nontemporal_store(vl, reinterpret_cast<f32x4 *>(dAl + i * ldda + c0));
            } else {
                dAh[i * ldda + c0] = d_h[0];
                dAl[i * ldda + c0] = d_l[0];
            }
        }
        if (WANT_DX) {
#pragma unroll
            for (int k = 0; k < COLS; ++k) {
                float ph, pl;
                ffd::mul22<false>(g_h, g_l, a_h[k], a_l[k], ph, pl);
                ffd::add22(acc[k].x, acc[k].y, ph, pl, acc[k].x, acc[k].y);
            }
        }
    };
    auto load_row = [&](int64_t i, float (&a_h)[COLS], float (&a_l)[COLS]) {
        if (WANT_DX) {
            if constexpr (COLS == 4) {
                const f32x4 vh = __builtin_nontemporal_load(reinterpret_cast<const f32x4 *>(Ah + i * lda + c0));
                const f32x4 vl = __builtin_nontemporal_load(reinterpret_cast<const f32x4 *>(Al + i * lda + c0));
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    a_h[k] = vh[k];
                    a_l[k] = vl[k];
                }
            } else {
                a_h[0] = Ah[i * lda + c0];
                a_l[0] = Al[i * lda + c0];
            }
        }
    };
    int64_t i = i0;
    for (; i + kRowPair <= i1; i += kRowPair) {
        float a_h[kRowPair][COLS], a_l[kRowPair][COLS];
#pragma unroll
        for (int p = 0; p < kRowPair; ++p)
            load_row(i + p, a_h[p], a_l[p]);
#pragma unroll
        for (int p = 0; p < kRowPair; ++p)
            row(i + p, a_h[p], a_l[p]);
    }
    for (; i < i1; ++i) {
        float a_h[COLS], a_l[COLS];
        load_row(i, a_h, a_l);
        row(i, a_h, a_l);
    }
    if (WANT_DX) {
#pragma unroll
        for (int k = 0; k < COLS; ++k)
            part[static_cast<int64_t>(blockIdx.y) * N + c0 + k] = acc[k];
    }
}

// dx_j = partial sums of column j added in band order.
// dx_j = sum over bands of the per-band partials, for 64 columns per
// workgroup: eight groups of threads take bands g, g + 8, ... (coalesced
// 512-byte rows of partials, several loads in flight per thread), then the
// eight group sums are added in a fixed tree through LDS.
constexpr int kCombineGroups = 8;

__global__ __launch_bounds__(64 * kCombineGroups) void matvec_bwd_combine(
    int64_t N, int64_t nbands, const float2 *__restrict__ part, float *__restrict__ dxh,
    float *__restrict__ dxl)
{
    __shared__ float2 sums[kCombineGroups][64];
    const int col = threadIdx.x & 63, grp = threadIdx.x >> 6;
    const int64_t j = static_cast<int64_t>(blockIdx.x) * 64 + col;
    float h = 0.0f, l = 0.0f;
    if (j < N) {
        int64_t b = grp;
        for (; b + 3 * kCombineGroups < nbands; b += 4 * kCombineGroups) {
            float2 p[4];
#pragma unroll
            for (int u = 0; u < 4; ++u)
                p[u] = part[(b + u * kCombineGroups) * N + j];
#pragma unroll
            for (int u = 0; u < 4; ++u)
                ffd::add22(h, l, p[u].x, p[u].y, h, l);
        }
        for (; b < nbands; b += kCombineGroups) {
            const float2 p = part[b * N + j];
            ffd::add22(h, l, p.x, p.y, h, l);
        }
    }
    sums[grp][col] = make_float2(h, l);
    __syncthreads();
#pragma unroll
    for (int w = kCombineGroups / 2; w >= 1; w >>= 1) {
        if (grp < w) {
            const float2 a = sums[grp][col], c = sums[grp + w][col];
            float rh, rl;
            ffd::add22(a.x, a.y, c.x, c.y, rh, rl);
            sums[grp][col] = make_float2(rh, rl);
        }
        __syncthreads();
    }
    if (grp == 0 && j < N) {
        dxh[j] = sums[0][col].x;
        dxl[j] = sums[0][col].y;
    }
}

// Plain backward, dx: one thread per column, rows in order.
__global__ __launch_bounds__(256) void matvec_bwd_plain_dx(
    int64_t M, int64_t N, const float *__restrict__ Ah, const float *__restrict__ Al, int64_t lda,
    const float *__restrict__ gh, const float *__restrict__ gl, float *__restrict__ dxh,
    float *__restrict__ dxl)
{
    const int64_t j = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (j >= N)
        return;
    float h = 0.0f, l = 0.0f;
    for (int64_t i = 0; i < M; ++i) {
        float ph, pl;
        ffd::mul22<false>(gh[i], gl[i], Ah[i * lda + j], Al[i * lda + j], ph, pl);
        ffd::add22(h, l, ph, pl, h, l);
    }
    dxh[j] = h;
    dxl[j] = l;
}

// Plain backward, dA: one thread per element.
__global__ __launch_bounds__(256) void matvec_bwd_plain_da(
    int64_t M, int64_t N, const float *__restrict__ xh, const float *__restrict__ xl,
    const float *__restrict__ gh, const float *__restrict__ gl, float *__restrict__ dAh,
    float *__restrict__ dAl, int64_t ldda)
{
    const int64_t j = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    const int64_t i = blockIdx.y;
    if (j >= N || i >= M)
        return;
    float h, l;
    ffd::mul22<false>(gh[i], gl[i], xh[j], xl[j], h, l);
    dAh[i * ldda + j] = h;
    dAl[i * ldda + j] = l;
}

// Backward pass of the single float-float dot s = sum x_i y_i for one
// upstream gradient g: dx_i = Mul22(g, y_i), dy_i = Mul22(g, x_i).  One
// workgroup of kDotBwdThreads per block of kDotBwdThreads * kDotBwdPer
// consecutive elements, in launch order; a thread loads all its
// lane-contiguous elements first, then computes and stores.  Small
// workgroups stream this pattern (four planes in, four out) fastest: 128
// threads by one element moved 6.2 TB/s at N = 2^28, against 6.0 for 128 by
// 2 and 5.35 for 1024 by 2; no block pays a per-block set-up here.
constexpr int kDotBwdThreads = 128;
constexpr int kDotBwdPer = 1;

__global__ __launch_bounds__(kDotBwdThreads) void dot_backward(const float *__restrict__ g_hi,
                                                    const float *__restrict__ g_lo,
                                                    const float *__restrict__ xh,
                                                    const float *__restrict__ xl,
                                                    const float *__restrict__ yh,
                                                    const float *__restrict__ yl,
                                                    float *__restrict__ dxh,
                                                    float *__restrict__ dxl,
                                                    float *__restrict__ dyh,
                                                    float *__restrict__ dyl, int64_t n)
{
    constexpr int kPer = kDotBwdPer;
    const float gh = g_hi[0], gl = g_lo[0];
    const int64_t b0 = static_cast<int64_t>(blockIdx.x) * (kDotBwdThreads * kPer) + threadIdx.x;
    const bool want_dx = dxh != nullptr, want_dy = dyh != nullptr;
    float ox[kPer], oxl[kPer], oy[kPer], oyl[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int64_t i = b0 + static_cast<int64_t>(kDotBwdThreads) * k;
        const bool in = i < n;
        ox[k] = (want_dy && in) ? xh[i] : 0.0f;
        oxl[k] = (want_dy && in) ? xl[i] : 0.0f;
        oy[k] = (want_dx && in) ? yh[i] : 0.0f;
        oyl[k] = (want_dx && in) ? yl[i] : 0.0f;
    }
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int64_t i = b0 + static_cast<int64_t>(kDotBwdThreads) * k;
        if (i >= n)
            break;
        float h, l;
        if (want_dx) {
            ffd::mul22<false>(gh, gl, oy[k], oyl[k], h, l);
            dxh[i] = h;
            dxl[i] = l;
        }
        if (want_dy) {
            ffd::mul22<false>(gh, gl, ox[k], oxl[k], h, l);
            dyh[i] = h;
            dyl[i] = l;
        }
    }
}

// Backward pass of the batched dot s_v = sum over vector v of x_i y_i:
// every element i of vector v gets dx_i = Mul22(g_v, y_i) and
// dy_i = Mul22(g_v, x_i); elements of no vector get zeros.  Two launches:
//   records   one thread per block of kBwdBlock consecutive elements: a
//             binary search over the clamped offsets for the vector owning
//             the block's first element, stored with that vector's gradient
//             and the next vector's start as one 16-byte record
//   gradients one workgroup per block, launched in order, so that the
//             resident workgroups sweep memory together: thread t takes
//             elements b0 + t + kBwdThreads k (each wavefront access is 256
//             contiguous bytes of a plane) and issues all its loads first,
//             then the block's record (one scalar load, on a counter of its
//             own); the vector starts inside a wavefront's range (usually
//             none) are walked, up to kBwdWalk of them, and past that (vectors
//             of a few elements) each lane searches its remaining elements'
//             owners
// Small blocks stream this pattern (two planes in, four out) fastest: a
// pass-through kernel moved 6.5 TB/s at 256 threads by one element, 6.25 at
// 128 by 1, 5.6 at 512 by 2 and 5.5 at 512 by 8 (438.9 M elements on
// MI355X).  A search per block at that size -- even one shared by the
// workgroup's wavefronts -- cost more than the access pattern gained (its
// dependent loads wait behind the streaming traffic), hence the records.
// 24 to 32 bytes per element and two Mul22: HBM-bound.
constexpr int kBwdThreads = 256;
constexpr int kBwdPer = 1;
constexpr int64_t kBwdBlock = static_cast<int64_t>(kBwdThreads) * kBwdPer;
constexpr int kBwdWalk = 8;
constexpr int kBwdRecordThreads = 256;

__device__ __forceinline__ int64_t clamped_offset(const int64_t *__restrict__ offsets, int64_t v,
                                                  int64_t total)
{
    const int64_t o = offsets[v];
    return o < 0 ? 0 : (o > total ? total : o);
}

// Number of vector starts at or before position p, minus one: the vector
// owning element p, in [-1, nvec] (-1: before the first vector, nvec: after
// the last).  With offsets out of order the result is still in that range.
__device__ __forceinline__ int64_t owner_of(const int64_t *__restrict__ offsets, int32_t nvec,
                                            int64_t total, int64_t p)
{
    int64_t lo = 0, hi = static_cast<int64_t>(nvec) + 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (clamped_offset(offsets, mid, total) <= p)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo - 1;
}

// Record of block b: x = the vector owning element b * kBwdBlock (-1 .. nvec),
// y, z = the bits of its gradient (zero when it is no vector), w = the start
// of the next vector relative to the block's first element, clipped to
// [0, INT32_MAX] (INT32_MAX: none within reach).
__global__ __launch_bounds__(kBwdRecordThreads) void dot_bwd_records(
    const float *__restrict__ g_hi, const float *__restrict__ g_lo,
    const int64_t *__restrict__ offsets, int32_t nvec, int64_t total, int64_t nblocks,
    int4 *__restrict__ records)
{
    const int64_t b = static_cast<int64_t>(blockIdx.x) * kBwdRecordThreads + threadIdx.x;
    if (b >= nblocks)
        return;
    const int64_t b0 = b * kBwdBlock;
    const int64_t v = owner_of(offsets, nvec, total, b0);
    const bool ok = v >= 0 && v < nvec;
    const float gh = ok ? g_hi[v] : 0.0f, gl = ok ? g_lo[v] : 0.0f;
    int64_t rel = INT32_MAX;
    if (v < nvec) {
        const int64_t o = clamped_offset(offsets, v + 1, total) - b0;
        rel = o < 0 ? 0 : (o < INT32_MAX ? o : INT32_MAX);
    }
    records[b] = make_int4(static_cast<int32_t>(v), __float_as_int(gh), __float_as_int(gl),
                           static_cast<int32_t>(rel));
}

template <bool XLO, bool YLO, bool DX, bool DY>
__global__ __launch_bounds__(kBwdThreads) void dot_batched_bwd(
    const float *__restrict__ g_hi, const float *__restrict__ g_lo,
    const int64_t *__restrict__ offsets, int32_t nvec, int64_t total,
    const int4 *__restrict__ records,
    const float *__restrict__ xh, const float *__restrict__ xl, const float *__restrict__ yh,
    const float *__restrict__ yl, float *__restrict__ dxh, float *__restrict__ dxl,
    float *__restrict__ dyh, float *__restrict__ dyl)
{
    const int t = threadIdx.x;
    const int64_t b0 = static_cast<int64_t>(blockIdx.x) * kBwdBlock;
    // all of this thread's operands first
    int64_t idx[kBwdPer];
    float ox[kBwdPer], oxl[kBwdPer], oy[kBwdPer], oyl[kBwdPer];
#pragma unroll
    for (int k = 0; k < kBwdPer; ++k) {
        const int64_t i = b0 + t + static_cast<int64_t>(kBwdThreads) * k;
        idx[k] = i;
        const bool in = i < total;
        ox[k] = (DY && in) ? xh[i] : 0.0f;
        oxl[k] = (DY && XLO && in) ? xl[i] : 0.0f;
        oy[k] = (DX && in) ? yh[i] : 0.0f;
        oyl[k] = (DX && YLO && in) ? yl[i] : 0.0f;
    }
    const int4 r = records[blockIdx.x];
    // the wavefront's first and last element, the same on every lane
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const int64_t w0 = b0 + 64 * wave;
    if (w0 >= total)
        return;
    const int64_t w_end = w0 + 63 + static_cast<int64_t>(kBwdThreads) * (kBwdPer - 1);
    const int64_t w_last = w_end < total ? w_end : total - 1;
    int64_t v = r.x;
    int64_t nxt = r.w == INT32_MAX ? INT64_MAX : b0 + r.w;
    bool has[kBwdPer];
    float gkh[kBwdPer], gkl[kBwdPer];
    {
        const bool ok = v >= 0 && v < nvec;
        const float gh = __int_as_float(r.y), gl = __int_as_float(r.z);
#pragma unroll
        for (int k = 0; k < kBwdPer; ++k) {
            has[k] = ok;
            gkh[k] = gh;
            gkl[k] = gl;
        }
    }
    // elements at or after the start nxt of vector v + 1 belong to it (or to
    // a later vector, found when its own start is reached)
    for (int step = 0; step < kBwdWalk && nxt <= w_last; ++step) {
        ++v;
        const bool ok = v < nvec;
        const float gh = ok ? g_hi[v] : 0.0f, gl = ok ? g_lo[v] : 0.0f;
#pragma unroll
        for (int k = 0; k < kBwdPer; ++k) {
            if (idx[k] >= nxt) {
                has[k] = ok;
                gkh[k] = gh;
                gkl[k] = gl;
            }
        }
        nxt = ok ? clamped_offset(offsets, v + 1, total) : INT64_MAX;
    }
    if (nxt <= w_last) {
        // more vector starts in this range than the walk takes
#pragma unroll
        for (int k = 0; k < kBwdPer; ++k) {
            if (idx[k] >= nxt && idx[k] < total) {
                const int64_t u = owner_of(offsets, nvec, total, idx[k]);
                has[k] = u >= 0 && u < nvec;
                gkh[k] = has[k] ? g_hi[u] : 0.0f;
                gkl[k] = has[k] ? g_lo[u] : 0.0f;
            }
        }
    }
#pragma unroll
    for (int k = 0; k < kBwdPer; ++k) {
        const int64_t i = idx[k];
        if (i >= total)
            break;
        float a = 0.0f, b = 0.0f, c = 0.0f, d = 0.0f;
        if (has[k]) {
            if (DX)
                ffd::mul22<false>(gkh[k], gkl[k], oy[k], oyl[k], a, b);
            if (DY)
                ffd::mul22<false>(gkh[k], gkl[k], ox[k], oxl[k], c, d);
        }
        if (DX) {
            dxh[i] = a;
            dxl[i] = b;
        }
        if (DY) {
            dyh[i] = c;
            dyl[i] = d;
        }
    }
}

bool all_aligned(std::initializer_list<const void *> ptrs, uintptr_t bytes)
{
    for (const void *p : ptrs)
        if (p && !ffh::aligned(p, bytes))
            return false;
    return true;
}

int64_t nbands_of(int64_t M) { return (M + kBandRows - 1) / kBandRows; }

} // namespace ffk

using namespace ffk;

extern "C" {

ff_status ff_matvec(int64_t M, int64_t N, const float *A_hi, const float *A_lo, int64_t lda,
                    const float *x_hi, const float *x_lo, float *y_hi, float *y_lo, int32_t algo,
                    void *stream)
{
    if (M < 0 || N < 0 || lda < N)
        return FF_ERR_SIZE;
    if (algo != FF_MATVEC_FAST && algo != FF_MATVEC_PLAIN)
        return FF_ERR_ARG;
    if (M == 0)
        return FF_OK;
    if (!y_hi || !y_lo || (N > 0 && (!A_hi || !A_lo || !x_hi || !x_lo)))
        return FF_ERR_NULL;
    if (!all_aligned({A_hi, A_lo, x_hi, x_lo, y_hi, y_lo}, 4))
        return FF_ERR_ALIGN;
    if (M > INT32_MAX)
        return FF_ERR_SIZE;
    hipStream_t st = ffh::as_stream(stream);
    if (algo == FF_MATVEC_PLAIN) {
        hipLaunchKernelGGL(matvec_plain, dim3(static_cast<unsigned>(ffh::cdiv(M, 256))), dim3(256),
                           0, st, M, N, A_hi, A_lo, lda, x_hi, x_lo, y_hi, y_lo);
    } else {
        const bool vec = all_aligned({A_hi, A_lo, x_hi, x_lo}, 16) && lda % 4 == 0;
        if (vec)
            hipLaunchKernelGGL((matvec_rows<kRowBlock, true>),
                               dim3(static_cast<unsigned>(ffh::cdiv(M, kRowsPerGroup))),
                               dim3(kRowBlock), 0, st, M, N, A_hi, A_lo, lda, x_hi, x_lo, y_hi,
                               y_lo);
        else
            hipLaunchKernelGGL((matvec_rows<kRowBlock, false>),
                               dim3(static_cast<unsigned>(ffh::cdiv(M, kRowsPerGroup))),
                               dim3(kRowBlock), 0, st, M, N, A_hi, A_lo, lda, x_hi, x_lo, y_hi,
                               y_lo);
    }
    return ffh::launch_status();
}

size_t ff_matvec_backward_workspace_size(int64_t M, int64_t N, int32_t algo)
{
    if (M < 0 || N < 0 || algo != FF_MATVEC_FAST)
        return 0;
    return static_cast<size_t>(nbands_of(M)) * static_cast<size_t>(N) * sizeof(float2);
}

ff_status ff_matvec_backward(int64_t M, int64_t N, const float *A_hi, const float *A_lo,
                             int64_t lda, const float *x_hi, const float *x_lo, const float *g_hi,
                             const float *g_lo, float *dA_hi, float *dA_lo, int64_t ldda,
                             float *dx_hi, float *dx_lo, int32_t algo, void *ws, size_t ws_bytes,
                             void *stream)
{
    if (M < 0 || N < 0 || lda < N)
        return FF_ERR_SIZE;
    if (algo != FF_MATVEC_FAST && algo != FF_MATVEC_PLAIN)
        return FF_ERR_ARG;
    const bool want_da = dA_hi || dA_lo;
    const bool want_dx = dx_hi || dx_lo;
    if ((want_da && (!dA_hi || !dA_lo)) || (want_dx && (!dx_hi || !dx_lo)))
        return FF_ERR_NULL;
    if (want_da && ldda < N)
        return FF_ERR_SIZE;
    if (N == 0 || (!want_da && !want_dx))
        return FF_OK;
    if ((M > 0 && (!g_hi || !g_lo)) || (want_da && (!x_hi || !x_lo)) ||
        (want_dx && M > 0 && (!A_hi || !A_lo)))
        return FF_ERR_NULL;
    if (!all_aligned({A_hi, A_lo, x_hi, x_lo, g_hi, g_lo, dA_hi, dA_lo, dx_hi, dx_lo}, 4))
        return FF_ERR_ALIGN;
    if (M > 65535 * kBandRows || M > INT32_MAX)
        return FF_ERR_SIZE;
    hipStream_t st = ffh::as_stream(stream);
    if (algo == FF_MATVEC_PLAIN) {
        if (want_da && M > 65535)
            return FF_ERR_SIZE;
        if (want_da && M > 0)
            hipLaunchKernelGGL(matvec_bwd_plain_da,
                               dim3(static_cast<unsigned>(ffh::cdiv(N, 256)), static_cast<unsigned>(M)),
                               dim3(256), 0, st, M, N, x_hi, x_lo, g_hi, g_lo, dA_hi, dA_lo, ldda);
        if (want_dx)
            hipLaunchKernelGGL(matvec_bwd_plain_dx, dim3(static_cast<unsigned>(ffh::cdiv(N, 256))),
                               dim3(256), 0, st, M, N, A_hi, A_lo, lda, g_hi, g_lo, dx_hi, dx_lo);
        return ffh::launch_status();
    }
    const int64_t nbands = nbands_of(M);
    if (want_dx && M > 0) {
        if (!ws)
            return FF_ERR_NULL;
        if (ws_bytes < ff_matvec_backward_workspace_size(M, N, algo))
            return FF_ERR_WORKSPACE;
        if (!ffh::aligned(ws, 16))
            return FF_ERR_ALIGN;
    }
    float2 *part = static_cast<float2 *>(ws);
    if (M > 0) {
        const bool vec = N % 4 == 0 && lda % 4 == 0 && (!want_da || ldda % 4 == 0) &&
                         all_aligned({A_hi, A_lo, dA_hi, dA_lo}, 16);
        const int cols = vec ? 4 : 1;
        const dim3 grid(static_cast<unsigned>(ffh::cdiv(N, int64_t(kColBlock) * cols)),
                        static_cast<unsigned>(nbands));
#define FF_BWD_LAUNCH(C, DA, DX)                                                               \
    hipLaunchKernelGGL((matvec_bwd_band<kColBlock, C, DA, DX>), grid, dim3(kColBlock), 0, st, M, \
                       N, A_hi, A_lo, lda, x_hi, x_lo, g_hi, g_lo, dA_hi, dA_lo, ldda, part)
        if (vec) {
            if (want_da && want_dx)
                FF_BWD_LAUNCH(4, true, true);
            else if (want_da)
                FF_BWD_LAUNCH(4, true, false);
            else
                FF_BWD_LAUNCH(4, false, true);
        } else {
            if (want_da && want_dx)
                FF_BWD_LAUNCH(1, true, true);
            else if (want_da)
                FF_BWD_LAUNCH(1, true, false);
            else
                FF_BWD_LAUNCH(1, false, true);
        }
#undef FF_BWD_LAUNCH
    }
    if (want_dx)
        hipLaunchKernelGGL(matvec_bwd_combine, dim3(static_cast<unsigned>(ffh::cdiv(N, 64))),
                           dim3(64 * kCombineGroups), 0, st, N, nbands, part, dx_hi, dx_lo);
    return ffh::launch_status();
}

ff_status ff_dot_backward(const float *g_hi, const float *g_lo, const float *x_hi,
                          const float *x_lo, const float *y_hi, const float *y_lo, float *dx_hi,
                          float *dx_lo, float *dy_hi, float *dy_lo, int64_t n, void *stream)
{
    if (n < 0)
        return FF_ERR_SIZE;
    const bool want_dx = dx_hi || dx_lo, want_dy = dy_hi || dy_lo;
    if ((want_dx && (!dx_hi || !dx_lo)) || (want_dy && (!dy_hi || !dy_lo)))
        return FF_ERR_NULL;
    if (n == 0 || (!want_dx && !want_dy))
        return FF_OK;
    if (!g_hi || !g_lo || (want_dx && (!y_hi || !y_lo)) || (want_dy && (!x_hi || !x_lo)))
        return FF_ERR_NULL;
    if (!all_aligned({g_hi, g_lo, x_hi, x_lo, y_hi, y_lo, dx_hi, dx_lo, dy_hi, dy_lo}, 4))
        return FF_ERR_ALIGN;
    const int64_t blocks = ffh::cdiv(n, int64_t(kDotBwdThreads) * kDotBwdPer);
    if (blocks > INT32_MAX)
        return FF_ERR_SIZE;
    hipLaunchKernelGGL(dot_backward, dim3(static_cast<unsigned>(blocks)), dim3(kDotBwdThreads), 0,
                       ffh::as_stream(stream), g_hi, g_lo, x_hi, x_lo, y_hi, y_lo,
                       want_dx ? dx_hi : nullptr, dx_lo, want_dy ? dy_hi : nullptr, dy_lo, n);
    return ffh::launch_status();
}

size_t ff_dot_batched_backward_workspace_size(int64_t total_len)
{
    if (total_len <= 0)
        return 0;
    return static_cast<size_t>(ffh::cdiv(total_len, kBwdBlock)) * sizeof(int4);
}

ff_status ff_dot_batched_backward(const float *g_hi, const float *g_lo, const int64_t *offsets,
                                  int32_t nvec, int64_t total_len, const float *x_hi,
                                  const float *x_lo, const float *y_hi, const float *y_lo,
                                  float *dx_hi, float *dx_lo, float *dy_hi, float *dy_lo,
                                  void *ws, size_t ws_bytes, void *stream)
{
    if (nvec < 0 || total_len < 0)
        return FF_ERR_SIZE;
    const bool want_dx = dx_hi || dx_lo, want_dy = dy_hi || dy_lo;
    if ((want_dx && (!dx_hi || !dx_lo)) || (want_dy && (!dy_hi || !dy_lo)))
        return FF_ERR_NULL;
    if (total_len == 0 || (!want_dx && !want_dy))
        return FF_OK;
    if (!offsets || (nvec > 0 && (!g_hi || !g_lo)) || (want_dx && !y_hi) || (want_dy && !x_hi))
        return FF_ERR_NULL;
    if (!ffh::aligned(offsets, 8) ||
        !all_aligned({g_hi, g_lo, x_hi, x_lo, y_hi, y_lo, dx_hi, dx_lo, dy_hi, dy_lo}, 4))
        return FF_ERR_ALIGN;
    const int64_t blocks = ffh::cdiv(total_len, kBwdBlock);
    if (blocks > INT32_MAX)
        return FF_ERR_SIZE;
    if (!ws || ws_bytes < ff_dot_batched_backward_workspace_size(total_len))
        return FF_ERR_WORKSPACE;
    if (!ffh::aligned(ws, 16))
        return FF_ERR_ALIGN;
    int4 *records = static_cast<int4 *>(ws);
    hipLaunchKernelGGL(dot_bwd_records,
                       dim3(static_cast<unsigned>(ffh::cdiv(blocks, int64_t(kBwdRecordThreads)))),
                       dim3(kBwdRecordThreads), 0, ffh::as_stream(stream), g_hi, g_lo, offsets,
                       nvec, total_len, blocks, records);
    const bool xlo = want_dy && x_lo, ylo = want_dx && y_lo;
    auto launch = [&](auto kernel) {
        hipLaunchKernelGGL(kernel, dim3(static_cast<unsigned>(blocks)), dim3(kBwdThreads), 0,
                           ffh::as_stream(stream), g_hi, g_lo, offsets, nvec, total_len,
                           static_cast<const int4 *>(records), x_hi, x_lo, y_hi, y_lo, dx_hi,
                           dx_lo, dy_hi, dy_lo);
    };
    // one instantiation per (low words present, outputs wanted)
    if (want_dx && want_dy) {
        if (xlo && ylo)
            launch(dot_batched_bwd<true, true, true, true>);
        else if (xlo)
            launch(dot_batched_bwd<true, false, true, true>);
        else if (ylo)
            launch(dot_batched_bwd<false, true, true, true>);
        else
            launch(dot_batched_bwd<false, false, true, true>);
    } else if (want_dx) {
        if (ylo)
            launch(dot_batched_bwd<false, true, true, false>);
        else
            launch(dot_batched_bwd<false, false, true, false>);
    } else {
        if (xlo)
            launch(dot_batched_bwd<true, false, false, true>);
        else
            launch(dot_batched_bwd<false, false, false, true>);
    }
    return ffh::launch_status();
}

} // extern "C"
