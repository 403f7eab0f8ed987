// ff_gemm.hip -- float-float matrix product C = A B (row-major planes).
//
// Two algorithms.
//
// FMA loop (the plain float-float GEMM): C_ij = Add22 accumulation, k
// ascending, of Mul22(A_ik, B_kj) -- section 4.1's operators applied term by
// term.  LDS-tiled (64 x 64 outputs per workgroup, 4 x 4 per thread), VALU
// bound: ~26 binary32 operations per multiply-add, no contraction.  Bit for
// bit the sequential definition.
//
// Sliced (the fast path; the paper has no GEMM): every entry of A and B is
// turned into a signed fixed-point integer relative to a power of two of its
// row (A) or column (B):
//     X_ik = round(A_ik 2^(P - e_i)),  2^e_i > max_k |A_ik|,  P = 8S - 2,
// and X is written as S = 7 signed 8-bit digits, X = sum_t d_t 256^(S-1-t).
// A_ik B_kj then expands into digit products d_t d'_u of weight
// 256^(2S-2-t-u); the pairs with t + u <= S - 1 (28 of 49) are kept.  Each
// pair is an integer GEMM on matrix cores:
//   * int8 digits, v_mfma_i32_32x32x32_i8, int32 accumulation;
//   * BF16 digits (integers |d| <= 128 are exact in BF16),
//     v_mfma_f32_32x32x16_bf16, FP32 accumulation folded every 128 k,
//     before any partial sum can exceed 2^24, into one exact 96-bit integer
//     per output, T += sum_D S_D 256^(6-D).
// All partial sums are exact integers, so the hardware's accumulation order
// does not matter.  Pairs on the same anti-diagonal D = t + u share one
// accumulator (same weight): |S_D| <= 7 K 2^14 < 2^31 for K <= 16384 (longer
// K is split into chunks summed with Add22).  The epilogue forms the exact
// 128-bit integer T = sum_D S_D 256^(6-D) and rounds it once to float-float:
//     C_ij ~ T 2^(e_i + f_j - 2P + 48).
// No binary64 arithmetic is used anywhere.  Error sources: rounding of X (at
// most one unit of 2^(e_i - P) per entry), the dropped pairs (< 2^-47 of
// 2^(e_i + f_j) K), and the final rounding (2^-48 |C_ij|).
//
// Data layout of the digit planes (workspace): for each slice t and tile of
// 64 rows of A (or 64 columns of B) by one K-stage of 32 bytes (32 int8 or 16
// BF16 digits: one matrix-core K-step), the 2 KiB tile is contiguous, so a
// stage is copied into LDS with straight 1 KiB wavefront loads; within a row
// the two 16-byte chunks are swapped on a row pattern (tile_swizzle) so that
// the operand reads hit distinct LDS banks.  B is stored transposed (K
// contiguous per column).
#include "ff_device.h"
#include "ff_host.h"

namespace ffk {

// ----------------------------------------------------------------- plain

constexpr int kPT = 64;   // plain tile: 64 x 64 outputs
constexpr int kPK = 16;   // k per LDS stage

__global__ __launch_bounds__(256) void gemm_fma_loop(int64_t M, int64_t N, int64_t K,
                                                     const float *__restrict__ Ah,
                                                     const float *__restrict__ Al, int64_t lda,
                                                     const float *__restrict__ Bh,
                                                     const float *__restrict__ Bl, int64_t ldb,
                                                     float *__restrict__ Ch,
                                                     float *__restrict__ Cl, int64_t ldc)
{
    __shared__ float sAh[kPK][kPT + 1], sAl[kPK][kPT + 1];
    __shared__ float sBh[kPK][kPT], sBl[kPK][kPT];
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    const int64_t i0 = static_cast<int64_t>(blockIdx.y) * kPT;
    const int64_t j0 = static_cast<int64_t>(blockIdx.x) * kPT;
    float ch[4][4], cl[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c)
            ch[r][c] = cl[r][c] = 0.0f;
    for (int64_t k0 = 0; k0 < K; k0 += kPK) {
        for (int e = threadIdx.x; e < kPT * kPK; e += 256) {
            const int r = e / kPK, c = e % kPK;
            const int64_t gi = i0 + r, gk = k0 + c;
            const bool ok = gi < M && gk < K;
            sAh[c][r] = ok ? Ah[gi * lda + gk] : 0.0f;
            sAl[c][r] = ok ? Al[gi * lda + gk] : 0.0f;
        }
        for (int e = threadIdx.x; e < kPK * kPT; e += 256) {
            const int r = e / kPT, c = e % kPT;
            const int64_t gk = k0 + r, gj = j0 + c;
            const bool ok = gk < K && gj < N;
            sBh[r][c] = ok ? Bh[gk * ldb + gj] : 0.0f;
            sBl[r][c] = ok ? Bl[gk * ldb + gj] : 0.0f;
        }
        __syncthreads();
        const int kmax = (K - k0 < kPK) ? static_cast<int>(K - k0) : kPK;
        for (int kk = 0; kk < kmax; ++kk) {
            float ah[4], al[4], bh[4], bl[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                ah[r] = sAh[kk][ty + 16 * r];
                al[r] = sAl[kk][ty + 16 * r];
            }
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                bh[c] = sBh[kk][tx + 16 * c];
                bl[c] = sBl[kk][tx + 16 * c];
            }
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    float ph, pl;
                    ffd::mul22<false>(ah[r], al[r], bh[c], bl[c], ph, pl);
                    ffd::add22(ch[r][c], cl[r][c], ph, pl, ch[r][c], cl[r][c]);
                }
        }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int64_t gi = i0 + ty + 16 * r, gj = j0 + tx + 16 * c;
            if (gi < M && gj < N) {
                Ch[gi * ldc + gj] = ch[r][c];
                Cl[gi * ldc + gj] = cl[r][c];
            }
        }
}

// ---------------------------------------------------------------- sliced

constexpr int kS = 7;                 // digits per operand
constexpr int kP = 8 * kS - 2;        // fixed-point bits: |X| <= 2^kP
constexpr int kTile = 64;             // rows (A) / columns (B) per tile
constexpr int kRowBytes = 32;         // digit bytes of one tile row per K-stage
constexpr int kTileBytes = kTile * kRowBytes;       // 2 KiB
constexpr int kEpiShift = 8 * (kS - 1) - 2 * kP;   // C = T 2^(e + f + kEpiShift)
constexpr int64_t kMaxKChunk = 16384; // int32 accumulators stay exact below this

typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef int i32x16 __attribute__((ext_vector_type(16)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __attribute__((address_space(3))) void *lds_void_ptr;
typedef const __attribute__((address_space(1))) void *global_void_ptr;

struct DigitsI8 {
    static constexpr int kEsize = 1;
    static constexpr int kStageK = kRowBytes;      // 32 digits: one i8 MFMA K-step
    static constexpr int kExtractStages = 0;       // int32 accumulation: never
};
struct DigitsBF16 {
    static constexpr int kEsize = 2;
    static constexpr int kStageK = kRowBytes / 2;  // 16 digits: one BF16 MFMA K-step
    static constexpr int kExtractStages = 8;       // drain FP32 every 128 k
};

__device__ __forceinline__ uint32_t f32_bits(float v) { return __float_as_uint(v); }

// Smallest e with |x| < 2^e for every x with |x| <= the value of bits ub.
__device__ __forceinline__ int exponent_bound(uint32_t ub)
{
    if (ub == 0)
        return 0;
    const int be = static_cast<int>(ub >> 23);
    return be == 0 ? -126 : be - 126;
}

// round(v * 2^scale_exp) as an integer (ties away from zero), saturating
// far outside the digit range.
__device__ __forceinline__ int64_t fixed_round(float v, int scale_exp)
{
    const uint32_t b = f32_bits(v);
    int be = static_cast<int>((b >> 23) & 255u);
    int64_t mant = b & 0x7fffffu;
    if (be == 0) {
        if (mant == 0)
            return 0;
        be = 1;
    } else {
        mant |= 0x800000;
    }
    const int sh = be - 150 + scale_exp;      // v = mant * 2^(be - 150)
    int64_t m;
    if (sh >= 0)
        m = mant << (sh < 38 ? sh : 38);
    else if (sh > -40)
        m = (mant + (int64_t(1) << (-sh - 1))) >> (-sh);
    else
        m = 0;
    return (b >> 31) ? -m : m;
}

// Digits of one float-float entry: d[0] most significant.
__device__ __forceinline__ void entry_digits(float hi, float lo, int e, int d[kS])
{
    const int se = kP - e;
    int64_t X = fixed_round(hi, se) + fixed_round(lo, se);
    const int64_t lim = int64_t(127) << (8 * (kS - 1));
    X = X > lim ? lim : (X < -lim ? -lim : X);
#pragma unroll
    for (int t = kS - 1; t >= 0; --t) {
        const int64_t dt = ((X + 128) & 255) - 128;
        d[t] = static_cast<int>(dt);
        X = (X - dt) >> 8;
    }
}

// Bit pattern of digit d in the plane's element type.
template <class Dg>
__device__ __forceinline__ uint32_t digit_bits(int d)
{
    if constexpr (Dg::kEsize == 1)
        return static_cast<uint32_t>(d) & 0xffu;
    else
        // |d| <= 128 has at most 8 significant bits: the BF16 pattern is the
        // upper half of the binary32 pattern, exactly.
        return f32_bits(static_cast<float>(d)) >> 16;
}

// Byte offset of (row, 16-byte chunk) inside a 2 KiB tile.  Rows are 32
// bytes; the two chunks of a row are swapped when bit 2 xor bit 3 of the row
// is set.  The operand reads take 16 consecutive rows at one logical chunk
// per 256-byte LDS cycle (64 banks of 4 bytes on gfx950): rows r and r + 8
// share a bank group unless their chunks differ, which this swizzle
// guarantees -- and 8-row groups stay conflict-free as well.
__device__ __forceinline__ int tile_swizzle(int row, int chunk)
{
    return row * kRowBytes + ((chunk ^ (((row >> 2) ^ (row >> 3)) & 1)) * 16);
}

__device__ __forceinline__ int64_t tile_base(int t, int bi, int bk, int nB, int nBK)
{
    return ((static_cast<int64_t>(t) * nB + bi) * nBK + bk) * kTileBytes;
}

__global__ __launch_bounds__(256) void fill_u32(uint32_t *p, int64_t n)
{
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * 256)
        p[i] = 0u;
}

// rowmax[i] = max_k |A_hi[i, k]| (as bits).  One wavefront per (row, 4096-k
// segment), 16-byte loads when the rows are 16-byte aligned; integer
// atomicMax, so the result does not depend on order.
template <bool VEC>
__global__ __launch_bounds__(256) void absmax_rows(int64_t M, int64_t K,
                                                   const float *__restrict__ Ah, int64_t lda,
                                                   uint32_t *__restrict__ rowmax)
{
    const int64_t row = static_cast<int64_t>(blockIdx.y) * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= M)
        return;
    const int64_t k0 = static_cast<int64_t>(blockIdx.x) * 4096;
    const int64_t k1 = (k0 + 4096 < K) ? k0 + 4096 : K;
    const float *a = Ah + row * lda;
    uint32_t m = 0;
    if (VEC) {
        const int64_t kv = k0 + ((k1 - k0) & ~int64_t(255));   // whole 256-entry steps
        for (int64_t k = k0 + 4 * lane; k < kv; k += 256) {
            const float4 v = *reinterpret_cast<const float4 *>(a + k);
            m = max(m, max(max(f32_bits(v.x) & 0x7fffffffu, f32_bits(v.y) & 0x7fffffffu),
                           max(f32_bits(v.z) & 0x7fffffffu, f32_bits(v.w) & 0x7fffffffu)));
        }
        for (int64_t k = kv + lane; k < k1; k += 64)
            m = max(m, f32_bits(a[k]) & 0x7fffffffu);
    } else {
        for (int64_t k = k0 + lane; k < k1; k += 64)
            m = max(m, f32_bits(a[k]) & 0x7fffffffu);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
        m = max(m, static_cast<uint32_t>(__shfl_xor(static_cast<int>(m), off, 64)));
    if (lane == 0 && m)
        atomicMax(&rowmax[row], m);
}

// colmax[j] = max_k |B_hi[k, j]|: thread per column, 64-row bands, eight
// independent loads in flight per thread.
__global__ __launch_bounds__(256) void absmax_cols(int64_t K, int64_t N,
                                                   const float *__restrict__ Bh, int64_t ldb,
                                                   uint32_t *__restrict__ colmax)
{
    const int64_t j = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (j >= N)
        return;
    const int64_t k0 = static_cast<int64_t>(blockIdx.y) * 64;
    const int64_t k1 = (k0 + 64 < K) ? k0 + 64 : K;
    uint32_t m[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int64_t k = k0;
    for (; k + 8 <= k1; k += 8) {
#pragma unroll
        for (int u = 0; u < 8; ++u)
            m[u] = max(m[u], f32_bits(Bh[(k + u) * ldb + j]) & 0x7fffffffu);
    }
    for (; k < k1; ++k)
        m[0] = max(m[0], f32_bits(Bh[k * ldb + j]) & 0x7fffffffu);
    uint32_t r = 0;
#pragma unroll
    for (int u = 0; u < 8; ++u)
        r = max(r, m[u]);
    if (r)
        atomicMax(&colmax[j], r);
}

// One 16-byte chunk of every slice for the entries (r, k0 .. k0 + per - 1)
// of a row (A) or column (B): packs the digits into four 32-bit words per
// slice and stores them at the swizzled tile position.
template <class Dg, class Load>
__device__ __forceinline__ void slice_chunk(Load load, bool row_ok, int64_t k0, int64_t K, int e,
                                            uint8_t *__restrict__ planes, int64_t plane_tile0,
                                            int64_t slice_stride, int in_tile)
{
    constexpr int kPer = 16 / Dg::kEsize;         // digits per chunk
    constexpr int kPerWord = 4 / Dg::kEsize;      // digits per 32-bit word
    uint32_t w[kS][4];
#pragma unroll
    for (int t = 0; t < kS; ++t)
#pragma unroll
        for (int q = 0; q < 4; ++q)
            w[t][q] = 0u;
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int64_t k = k0 + q;
        int d[kS];
        if (row_ok && k < K) {
            float hi, lo;
            load(k, hi, lo);
            entry_digits(hi, lo, e, d);
        } else {
#pragma unroll
            for (int t = 0; t < kS; ++t)
                d[t] = 0;
        }
#pragma unroll
        for (int t = 0; t < kS; ++t)
            w[t][q / kPerWord] |= digit_bits<Dg>(d[t]) << (8 * Dg::kEsize * (q % kPerWord));
    }
#pragma unroll
    for (int t = 0; t < kS; ++t)
        *reinterpret_cast<uint4 *>(planes + plane_tile0 + t * slice_stride + in_tile) =
            make_uint4(w[t][0], w[t][1], w[t][2], w[t][3]);
}

// A digit planes: workgroup = (64-row tile, K stage), 128 threads, thread =
// (row, chunk).
// Digit planes of A.  A workgroup covers 32 rows by 8 consecutive 16-byte
// chunks (4 K-stages) of each row; a thread converts one chunk: kPer
// consecutive entries of its row, read with 16-byte loads when the rows are
// 16-byte aligned (adjacent threads read adjacent 64- or 32-byte pieces of
// the row).  Rows at or beyond M and entries at or beyond K give zero
// digits (the tiles are padded).
template <class Dg>
__global__ __launch_bounds__(256) void slice_rows(int64_t M, int64_t K,
                                                  const float *__restrict__ Ah,
                                                  const float *__restrict__ Al, int64_t lda,
                                                  const uint32_t *__restrict__ rowmax, int nBI,
                                                  int nBK, uint8_t *__restrict__ planes, int vec)
{
    constexpr int kPer = 16 / Dg::kEsize;                 // entries per chunk
    constexpr int kChunks = Dg::kStageK / kPer;           // chunks per K-stage (2)
    const int c = threadIdx.x & 7;
    const int64_t i = static_cast<int64_t>(blockIdx.y) * 32 + (threadIdx.x >> 3);
    const int64_t kc = static_cast<int64_t>(blockIdx.x) * 8 + c;
    const int bk = static_cast<int>(kc / kChunks), chunk = static_cast<int>(kc % kChunks);
    if (bk >= nBK || i >= static_cast<int64_t>(nBI) * kTile)
        return;
    const bool ok = i < M;
    const int e = ok ? exponent_bound(rowmax[i]) : 0;
    const int64_t k0 = kc * kPer;
    const int bi = static_cast<int>(i / kTile), row = static_cast<int>(i % kTile);
    const int64_t slice_stride = static_cast<int64_t>(nBI) * nBK * kTileBytes;
    const int in_tile = tile_swizzle(row, chunk);
    if (vec && ok && k0 + kPer <= K) {
        float hv[kPer], lv[kPer];
#pragma unroll
        for (int q = 0; q < kPer; q += 4) {
            const float4 h4 = *reinterpret_cast<const float4 *>(Ah + i * lda + k0 + q);
            const float4 l4 = *reinterpret_cast<const float4 *>(Al + i * lda + k0 + q);
            hv[q] = h4.x; hv[q + 1] = h4.y; hv[q + 2] = h4.z; hv[q + 3] = h4.w;
            lv[q] = l4.x; lv[q + 1] = l4.y; lv[q + 2] = l4.z; lv[q + 3] = l4.w;
        }
        auto load = [&](int64_t k, float &hi, float &lo) {
            hi = hv[k - k0];
            lo = lv[k - k0];
        };
        slice_chunk<Dg>(load, true, k0, K, e, planes, tile_base(0, bi, bk, nBI, nBK),
                        slice_stride, in_tile);
    } else {
        auto load = [&](int64_t k, float &hi, float &lo) {
            hi = Ah[i * lda + k];
            lo = Al[i * lda + k];
        };
        slice_chunk<Dg>(load, ok, k0, K, e, planes, tile_base(0, bi, bk, nBI, nBK),
                        slice_stride, in_tile);
    }
}
template <class Dg>
__global__ __launch_bounds__(128) void slice_cols(int64_t K, int64_t N,
                                                  const float *__restrict__ Bh,
                                                  const float *__restrict__ Bl, int64_t ldb,
                                                  const uint32_t *__restrict__ colmax, int nBJ,
                                                  int nBK, uint8_t *__restrict__ planes)
{
    const int bk = blockIdx.x, bj = blockIdx.y;
    const int col = threadIdx.x & 63, chunk = threadIdx.x >> 6;
    const int64_t j = static_cast<int64_t>(bj) * kTile + col;
    const bool ok = j < N;
    const int e = ok ? exponent_bound(colmax[j]) : 0;
    const int64_t k0 = static_cast<int64_t>(bk) * Dg::kStageK + chunk * (16 / Dg::kEsize);
    auto load = [&](int64_t k, float &hi, float &lo) {
        hi = Bh[k * ldb + j];
        lo = Bl[k * ldb + j];
    };
    slice_chunk<Dg>(load, ok, k0, K, e, planes, tile_base(0, bj, bk, nBJ, nBK),
                    static_cast<int64_t>(nBJ) * nBK * kTileBytes, tile_swizzle(col, chunk));
}

// Round the integer t to 24 bits, nearest-even: t ~ mant 2^E (E >= 0).
__device__ __forceinline__ void round_i128(__int128 t, int &neg, uint32_t &mant, int &E)
{
    neg = t < 0;
    const unsigned __int128 u = neg ? static_cast<unsigned __int128>(-t)
                                    : static_cast<unsigned __int128>(t);
    const uint64_t hi = static_cast<uint64_t>(u >> 64), lo = static_cast<uint64_t>(u);
    const int nbits = hi ? 128 - __builtin_clzll(hi) : (lo ? 64 - __builtin_clzll(lo) : 0);
    if (nbits <= 24) {
        mant = static_cast<uint32_t>(lo);
        E = 0;
        return;
    }
    int sh = nbits - 24;
    unsigned __int128 m = u >> sh;
    const unsigned __int128 rem = u - (m << sh);
    const unsigned __int128 half = static_cast<unsigned __int128>(1) << (sh - 1);
    if (rem > half || (rem == half && (m & 1))) {
        m += 1;
        if (m >> 24) {
            m >>= 1;
            sh += 1;
        }
    }
    mant = static_cast<uint32_t>(m);
    E = sh;
}

// (hi, lo) = (RN(T), RN(T - RN(T))) * 2^scale.
__device__ __forceinline__ void i128_to_ff(__int128 T, int scale, float &hi, float &lo)
{
    int neg, E;
    uint32_t mant;
    round_i128(T, neg, mant, E);
    const __int128 top = static_cast<__int128>(mant) << E;
    const __int128 rem = T - (neg ? -top : top);
    const float h = __builtin_ldexpf(static_cast<float>(mant), E + scale);
    hi = neg ? -h : h;
    int rneg, rE;
    uint32_t rmant;
    round_i128(rem, rneg, rmant, rE);
    const float l = __builtin_ldexpf(static_cast<float>(rmant), rE + scale);
    lo = rneg ? -l : l;
}

__device__ __forceinline__ i32x16 mma(const uint4 &a, const uint4 &b, const i32x16 &c, DigitsI8)
{
    return __builtin_amdgcn_mfma_i32_32x32x32_i8(*reinterpret_cast<const i32x4 *>(&a),
                                                 *reinterpret_cast<const i32x4 *>(&b), c, 0, 0,
                                                 0);
}
__device__ __forceinline__ f32x16 mma(const uint4 &a, const uint4 &b, const f32x16 &c,
                                      DigitsBF16)
{
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(*reinterpret_cast<const bf16x8 *>(&a),
                                                   *reinterpret_cast<const bf16x8 *>(&b), c, 0,
                                                   0, 0);
}

template <class Dg> struct AccOf;
template <> struct AccOf<DigitsI8> { using T = i32x16; };
template <> struct AccOf<DigitsBF16> { using T = f32x16; };

// One LDS slot of the stage ring.  Each slot is a distinct LDS variable, so
// the compiler can tell a slot being read from one being filled by DMA.
template <int BYTES, int I>
__device__ __forceinline__ uint8_t *lds_slot()
{
    __shared__ uint4 slot[BYTES / 16];
    return reinterpret_cast<uint8_t *>(slot);
}

// Epilogue of a wavefront's 32 x 32 block: lane holds
// C[8*(r/4) + 4*(lane/32) + (r%4)][lane%32] for r = 0..15 as S diagonal sums;
// T = sum_D S_D 256^(S-1-D) is formed exactly and rounded once to
// float-float, then scaled by the row and column powers of two (and added
// to C with Add22 for the later K-chunks).
template <class Dg, int WM, int WN, class Acc>
__device__ __forceinline__ void store_block(const Acc (&acc)[kS], const i32x16 (&iacc)[kS],
                                            int64_t M, int64_t N, int bi, int bj, int wm, int wn,
                                            int lane, const uint32_t *__restrict__ rowmax,
                                            const uint32_t *__restrict__ colmax,
                                            float *__restrict__ Ch, float *__restrict__ Cl,
                                            int64_t ldc, int accumulate)
{
    const int64_t j = static_cast<int64_t>(bj) * (32 * WN) + wn * 32 + (lane & 31);
    const int fj = j < N ? exponent_bound(colmax[j]) : 0;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int m = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int64_t i = static_cast<int64_t>(bi) * (32 * WM) + wm * 32 + m;
        if (i >= M || j >= N)
            continue;
        __int128 T = 0;
#pragma unroll
        for (int d = 0; d < kS; ++d) {
            int sd;
            if constexpr (Dg::kExtractStages > 0)
                sd = iacc[d][r];
            else
                sd = acc[d][r];
            T = (T << 8) + static_cast<__int128>(sd);
        }
        float h, l;
        i128_to_ff(T, exponent_bound(rowmax[i]) + fj + kEpiShift, h, l);
        if (accumulate)
            ffd::add22(Ch[i * ldc + j], Cl[i * ldc + j], h, l, h, l);
        Ch[i * ldc + j] = h;
        Cl[i * ldc + j] = l;
    }
}

// As store_block, with T already formed (96-bit two's complement words).
template <int WM, int WN>
__device__ __forceinline__ void store_block_t96(const uint32_t (&t96)[16][3], int64_t M,
                                                int64_t N, int bi, int bj, int wm, int wn,
                                                int lane, const uint32_t *__restrict__ rowmax,
                                                const uint32_t *__restrict__ colmax,
                                                float *__restrict__ Ch, float *__restrict__ Cl,
                                                int64_t ldc, int accumulate)
{
    const int64_t j = static_cast<int64_t>(bj) * (32 * WN) + wn * 32 + (lane & 31);
    const int fj = j < N ? exponent_bound(colmax[j]) : 0;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int m = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int64_t i = static_cast<int64_t>(bi) * (32 * WM) + wm * 32 + m;
        if (i >= M || j >= N)
            continue;
        __int128 T = static_cast<__int128>(static_cast<int32_t>(t96[r][2]));
        T = (T << 64) | (static_cast<__int128>(t96[r][1]) << 32) |
            static_cast<__int128>(t96[r][0]);
        float h, l;
        i128_to_ff(T, exponent_bound(rowmax[i]) + fj + kEpiShift, h, l);
        if (accumulate)
            ffd::add22(Ch[i * ldc + j], Cl[i * ldc + j], h, l, h, l);
        Ch[i * ldc + j] = h;
        Cl[i * ldc + j] = l;
    }
}

// Launch shape of the sliced product: WM x WN = 4 x 2 wavefronts (2 per
// SIMD), each owning a 32 x 32 block of C as S diagonal accumulators, for a
// 128 x 64 block per workgroup; a ring of 3 K-stages of 42 KiB in LDS.
template <class Dg> struct SlicedShape {
    static constexpr int WM = 4, WN = 2;
};

// s_waitcnt immediate that waits until at most n vector-memory operations of
// this wavefront are outstanding (export and LDS counters left at maximum).
constexpr int vmcnt_imm(int n) { return (n & 15) | ((n >> 4) << 14) | (7 << 4) | (15 << 8); }

// Workgroup barrier without a memory fence: the LDS DMA of the next stage
// keeps flying across it (a __syncthreads fence would wait for it).  The
// "memory" clobber keeps the compiler from moving LDS accesses across.
__device__ __forceinline__ void barrier_no_fence() { asm volatile("s_barrier" ::: "memory"); }

// s_waitcnt immediate that waits until at most n LDS operations of this
// wavefront are outstanding.
constexpr int lgkmcnt_imm(int n) { return 15 | (3 << 14) | (7 << 4) | ((n & 15) << 8); }

// The sliced product with a ping-pong schedule (int8 digits, and BF16 digits
// with exact 96-bit per-output drains).  The 8 wavefronts form two
// groups (waves 0-3 and 4-7: one of each on every SIMD) that run half a
// K-stage apart: while one group reads a stage's fragments from LDS, the
// other runs the MFMAs of the fragments it read before, so the LDS reads
// land under the matrix-core work of the other group.  Two barriers per
// stage k:
//   phase 1: group 0 reads stage k, then issues its share of the DMA of
//            stage k + 2;  group 1 multiplies stage k - 1
//   phase 2: group 0 multiplies stage k;  group 1 reads stage k, then
//            issues its share of the DMA of stage k + 2
// Three LDS slots: the DMA of stage k + 2 fills the slot of stage k - 1,
// which both groups finished reading before the last barrier (group 1
// waits for its reads to land before that barrier).  A wavefront waits for
// its previous DMA share at the start of its next read phase, one stage
// after issuing it, and so before the barrier that precedes any read of it.
template <class Dg, int WM, int WN>
__global__ __launch_bounds__(64 * WM * WN, 2) void gemm_sliced_pp(
    int64_t M, int64_t N, int nBI, int nBJ, int nBK, int bk0, int bk1,
    const uint8_t *__restrict__ Ap, const uint8_t *__restrict__ Bp,
    const uint32_t *__restrict__ rowmax, const uint32_t *__restrict__ colmax,
    float *__restrict__ Ch, float *__restrict__ Cl, int64_t ldc, int accumulate)
{
    using Acc = typename AccOf<Dg>::T;
    constexpr bool kDrain = Dg::kExtractStages > 0;
    constexpr int kWaves = WM * WN;
    static_assert(kWaves == 8, "two groups of four wavefronts");
    constexpr int kTA = WM / 2, kTB = WN / 2;
    constexpr int kSlotBytes = kS * (kTA + kTB) * kTileBytes;
    constexpr int kHalves = 2 * kS * (kTA + kTB);
    constexpr int kQ = kHalves / kWaves, kR = kHalves % kWaves;
    uint8_t *const slot0 = lds_slot<kSlotBytes, 0>();
    uint8_t *const slot1 = lds_slot<kSlotBytes, 1>();
    uint8_t *const slot2 = lds_slot<kSlotBytes, 2>();

    const int bj = blockIdx.x, bi = blockIdx.y;
    const int tid = threadIdx.x, lane = tid & 63;
    // wavefront index as a scalar, so that the group test is a uniform branch
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave / WN, wn = wave % WN;
    const int64_t a_slice = static_cast<int64_t>(nBI) * nBK * kTileBytes;
    const int64_t b_slice = static_cast<int64_t>(nBJ) * nBK * kTileBytes;

    Acc acc[kS];
#pragma unroll
    for (int d = 0; d < kS; ++d)
#pragma unroll
        for (int r = 0; r < 16; ++r)
            acc[d][r] = 0;
    // BF16 digits: the FP32 stage sums are exact only up to 2^24, so every
    // kExtractStages stages they are folded into one exact integer per
    // output, T += sum_D S_D 256^(S-1-D), kept as 96 bits (three words,
    // two's complement): |T| < 7 K 2^14 2^49 < 2^78 for K <= 16384.
    uint32_t t96[kDrain ? 16 : 1][3];
#pragma unroll
    for (int r = 0; r < (kDrain ? 16 : 1); ++r)
        t96[r][0] = t96[r][1] = t96[r][2] = 0u;
    auto drain = [&]() {
        if constexpr (kDrain) {
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                __int128 t = 0;
#pragma unroll
                for (int d = 0; d < kS; ++d)
                    t = (t << 8) + static_cast<__int128>(static_cast<int>(acc[d][r]));
                __int128 T = static_cast<__int128>(static_cast<int32_t>(t96[r][2]));
                T = (T << 64) | (static_cast<__int128>(t96[r][1]) << 32) |
                    static_cast<__int128>(t96[r][0]);
                T += t;
                t96[r][0] = static_cast<uint32_t>(T);
                t96[r][1] = static_cast<uint32_t>(T >> 32);
                t96[r][2] = static_cast<uint32_t>(T >> 64);
            }
#pragma unroll
            for (int d = 0; d < kS; ++d)
#pragma unroll
                for (int r = 0; r < 16; ++r)
                    acc[d][r] = 0.0f;
        }
    };
    auto drain_due = [&](int bk) {
        return kDrain && ((bk - bk0 + 1) % (kDrain ? Dg::kExtractStages : 1) == 0 || bk + 1 == bk1);
    };

    auto fetch = [&](int bk, uint8_t *slot) {
#pragma unroll
        for (int j = 0; j < kQ + (kR ? 1 : 0); ++j) {
            const int h = wave + j * kWaves;
            if (h < kHalves) {
                const int tile = h >> 1, half = h & 1;
                const uint8_t *src;
                if (tile < kS * kTA) {
                    const int t = tile / kTA, tt = tile % kTA;
                    src = Ap + t * a_slice + tile_base(0, bi * kTA + tt, bk, nBI, nBK);
                } else {
                    const int tb = tile - kS * kTA;
                    const int t = tb / kTB, tt = tb % kTB;
                    src = Bp + t * b_slice + tile_base(0, bj * kTB + tt, bk, nBJ, nBK);
                }
                src += half * 1024 + lane * 16;
                uint8_t *dst = slot + tile * kTileBytes + half * 1024;
                __builtin_amdgcn_global_load_lds((global_void_ptr)(const void *)src,
                                                 (lds_void_ptr)(void *)dst, 16, 0, 0);
            }
        }
    };

    const int ta = wm >> 1, rla = 32 * (wm & 1) + (lane & 31);
    const int tb = wn >> 1, rlb = 32 * (wn & 1) + (lane & 31);
    const int oa = ta * kTileBytes + tile_swizzle(rla, lane >> 5);
    const int ob = kS * kTA * kTileBytes + tb * kTileBytes + tile_swizzle(rlb, lane >> 5);

    uint4 fa[kS], fb[kS];
    auto read_frags = [&](const uint8_t *slot) {
        fb[0] = *reinterpret_cast<const uint4 *>(slot + ob);
#pragma unroll
        for (int t = 0; t < kS; ++t)
            fa[t] = *reinterpret_cast<const uint4 *>(slot + t * kTA * kTileBytes + oa);
#pragma unroll
        for (int u = 1; u < kS; ++u)
            fb[u] = *reinterpret_cast<const uint4 *>(slot + u * kTB * kTileBytes + ob);
    };
    // The 28 digit pairs (t, u) in an order that keeps the updates of each
    // diagonal accumulator t + u at least three instructions apart, so that
    // no MFMA waits for the one before it (in a phase the SIMD's other
    // wavefront issues no MFMAs that could fill such a gap).
    auto mfmas = [&]() {
        constexpr int kOrder[28][2] = {
            {0, 6}, {0, 5}, {0, 4}, {0, 3}, {1, 5}, {1, 4}, {1, 3}, {1, 2}, {2, 4}, {2, 3},
            {2, 2}, {2, 1}, {3, 3}, {3, 2}, {3, 1}, {3, 0}, {4, 2}, {4, 1}, {4, 0}, {0, 2},
            {5, 1}, {5, 0}, {1, 1}, {0, 1}, {6, 0}, {2, 0}, {1, 0}, {0, 0}};
        static_assert(kS == 7, "the order lists the 28 pairs of 7 digits");
#pragma unroll
        for (int q = 0; q < 28; ++q) {
            const int t = kOrder[q][0], u = kOrder[q][1];
            acc[t + u] = mma(fa[t], fb[u], acc[t + u], Dg{});
            if ((q & 3) == 3)
                __builtin_amdgcn_sched_barrier(0);
        }
    };
    // A read phase: this wavefront's previous DMA share (stage bk + 1) has
    // landed, the fragments of stage bk are read, and the share of stage
    // bk + 2 goes out.
    auto read_phase = [&](const uint8_t *slot, uint8_t *dma_slot, int bk) {
        __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));
        read_frags(slot);
        __builtin_amdgcn_sched_barrier(0);
        if (bk + 2 < bk1)
            fetch(bk + 2, dma_slot);
        __builtin_amdgcn_sched_barrier(0);
    };

    // stages bk0 and bk0 + 1 in flight; stage bk0 landed everywhere
    if (bk0 < bk1)
        fetch(bk0, slot0);
    if (bk0 + 1 < bk1)
        fetch(bk0 + 1, slot1);
    if (bk0 + 1 < bk1) {
        if (kR != 0 && wave < kR)
            __builtin_amdgcn_s_waitcnt(vmcnt_imm(kQ + 1));
        else
            __builtin_amdgcn_s_waitcnt(vmcnt_imm(kQ));
    } else {
        __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));
    }
    barrier_no_fence();

    if (wave < 4) {
        auto stage0 = [&](const uint8_t *slot, uint8_t *dma_slot, int bk) {
            read_phase(slot, dma_slot, bk);
            barrier_no_fence();
            mfmas();
            if (drain_due(bk))
                drain();
            __builtin_amdgcn_sched_barrier(0);
            barrier_no_fence();
        };
        for (int bk = bk0; bk < bk1; bk += 3) {
            stage0(slot0, slot2, bk);
            if (bk + 1 < bk1)
                stage0(slot1, slot0, bk + 1);
            if (bk + 2 < bk1)
                stage0(slot2, slot1, bk + 2);
        }
    } else {
        auto stage1 = [&](const uint8_t *slot, uint8_t *dma_slot, int bk) {
            if (bk > bk0) {
                mfmas();
                if (drain_due(bk - 1))
                    drain();
            }
            __builtin_amdgcn_sched_barrier(0);
            barrier_no_fence();
            read_phase(slot, dma_slot, bk);
            // reads landed before the barrier: the DMA of the next stage
            // overwrites the slot of the stage before this one
            __builtin_amdgcn_s_waitcnt(lgkmcnt_imm(0));
            barrier_no_fence();
        };
        for (int bk = bk0; bk < bk1; bk += 3) {
            stage1(slot0, slot2, bk);
            if (bk + 1 < bk1)
                stage1(slot1, slot0, bk + 1);
            if (bk + 2 < bk1)
                stage1(slot2, slot1, bk + 2);
        }
        if (bk0 < bk1) {
            mfmas();   // the last stage
            drain();   // (always due after the last stage)
        }
    }
    __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));
    if constexpr (kDrain)
        store_block_t96<WM, WN>(t96, M, N, bi, bj, wm, wn, lane, rowmax, colmax, Ch, Cl, ldc,
                                accumulate);
    else
        store_block<Dg, WM, WN>(acc, acc, M, N, bi, bj, wm, wn, lane, rowmax, colmax, Ch, Cl,
                                ldc, accumulate);
}

struct SliceGeom {
    int nBI, nBJ, nBK;
    size_t plane_a, plane_b;   // bytes of all A / B digit planes
    size_t off_rowmax, off_colmax, off_a, off_b, total;
};

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

inline SliceGeom slice_geom(int64_t M, int64_t N, int64_t K, int stage_k)
{
    SliceGeom g;
    // tile counts padded to even numbers: a workgroup covers up to two
    // 64-row (or 64-column) tiles; the padding tiles hold zero digits
    g.nBI = 2 * static_cast<int>((M + 2 * kTile - 1) / (2 * kTile));
    g.nBJ = 2 * static_cast<int>((N + 2 * kTile - 1) / (2 * kTile));
    g.nBK = static_cast<int>((K + stage_k - 1) / stage_k);
    g.plane_a = static_cast<size_t>(kS) * g.nBI * g.nBK * kTileBytes;
    g.plane_b = static_cast<size_t>(kS) * g.nBJ * g.nBK * kTileBytes;
    g.off_rowmax = 0;
    g.off_colmax = align256(sizeof(uint32_t) * M);
    g.off_a = g.off_colmax + align256(sizeof(uint32_t) * N);
    g.off_b = g.off_a + align256(g.plane_a);
    g.total = g.off_b + align256(g.plane_b);
    return g;
}

template <class Dg>
ff_status sliced_gemm(int64_t M, int64_t N, int64_t K, const float *Ah, const float *Al,
                      int64_t lda, const float *Bh, const float *Bl, int64_t ldb, float *Ch,
                      float *Cl, int64_t ldc, void *ws, size_t ws_bytes, hipStream_t st)
{
    const SliceGeom g = slice_geom(M, N, K, Dg::kStageK);
    if (!ws)
        return FF_ERR_NULL;
    if (ws_bytes < g.total)
        return FF_ERR_WORKSPACE;
    if (!ffh::aligned(ws, 256))
        return FF_ERR_ALIGN;
    if (g.nBI > 32767 || g.nBJ > 65535 || ffh::cdiv(M, 4) > 65535 || ffh::cdiv(K, 64) > 65535)
        return FF_ERR_SIZE;
    char *base = static_cast<char *>(ws);
    uint32_t *rowmax = reinterpret_cast<uint32_t *>(base + g.off_rowmax);
    uint32_t *colmax = reinterpret_cast<uint32_t *>(base + g.off_colmax);
    uint8_t *Ap = reinterpret_cast<uint8_t *>(base + g.off_a);
    uint8_t *Bp = reinterpret_cast<uint8_t *>(base + g.off_b);

    const int64_t nfill = static_cast<int64_t>(g.off_a / sizeof(uint32_t));
    const int64_t fill_blocks = ffh::cdiv(nfill, 256);
    hipLaunchKernelGGL(fill_u32, dim3(static_cast<unsigned>(fill_blocks < 4096 ? fill_blocks : 4096)),
                       dim3(256), 0, st, rowmax, nfill);
    if (K > 0) {
        const bool rows_vec = lda % 4 == 0 && ffh::aligned(Ah, 16) && ffh::aligned(Al, 16);
        const dim3 rgrid(static_cast<unsigned>(ffh::cdiv(K, 4096)),
                         static_cast<unsigned>(ffh::cdiv(M, 4)));
        if (rows_vec)
            hipLaunchKernelGGL(absmax_rows<true>, rgrid, dim3(256), 0, st, M, K, Ah, lda, rowmax);
        else
            hipLaunchKernelGGL(absmax_rows<false>, rgrid, dim3(256), 0, st, M, K, Ah, lda, rowmax);
        hipLaunchKernelGGL(absmax_cols,
                           dim3(static_cast<unsigned>(ffh::cdiv(N, 256)),
                                static_cast<unsigned>(ffh::cdiv(K, 64))),
                           dim3(256), 0, st, K, N, Bh, ldb, colmax);
        constexpr int kChunks = Dg::kStageK / (16 / Dg::kEsize);
        hipLaunchKernelGGL((slice_rows<Dg>),
                           dim3(static_cast<unsigned>(ffh::cdiv(static_cast<int64_t>(g.nBK) * kChunks, 8)),
                                static_cast<unsigned>(g.nBI * (kTile / 32))),
                           dim3(256), 0, st, M, K, Ah, Al, lda, rowmax, g.nBI, g.nBK, Ap,
                           rows_vec ? 1 : 0);
        hipLaunchKernelGGL((slice_cols<Dg>), dim3(g.nBK, g.nBJ), dim3(128), 0, st, K, N, Bh, Bl,
                           ldb, colmax, g.nBJ, g.nBK, Bp);
    }
    using Sh = SlicedShape<Dg>;
    const int stages_per_chunk = static_cast<int>(kMaxKChunk / Dg::kStageK);
    const dim3 grid(static_cast<unsigned>(g.nBJ / (Sh::WN / 2)),
                    static_cast<unsigned>(g.nBI / (Sh::WM / 2)));
    int bk0 = 0;
    do {
        const int bk1 = (bk0 + stages_per_chunk < g.nBK) ? bk0 + stages_per_chunk : g.nBK;
        hipLaunchKernelGGL((gemm_sliced_pp<Dg, Sh::WM, Sh::WN>), grid, dim3(64 * Sh::WM * Sh::WN),
                           0, st, M, N, g.nBI, g.nBJ, g.nBK, bk0, bk1, Ap, Bp, rowmax, colmax, Ch,
                           Cl, ldc, bk0 > 0 ? 1 : 0);
        bk0 = bk1;
    } while (bk0 < g.nBK);
    return ffh::launch_status();
}

} // namespace ffk

using namespace ffk;

extern "C" {

size_t ff_gemm_workspace_size(int64_t M, int64_t N, int64_t K, int32_t algo)
{
    if (M < 0 || N < 0 || K < 0)
        return 0;
    switch (algo) {
    case FF_GEMM_FMA_LOOP: return 0;
    case FF_GEMM_SLICED_BF16: return slice_geom(M, N, K, DigitsBF16::kStageK).total;
    case FF_GEMM_SLICED_I8: return slice_geom(M, N, K, DigitsI8::kStageK).total;
    default: return 0;
    }
}

ff_status ff_gemm(int64_t M, int64_t N, int64_t K, const float *A_hi, const float *A_lo,
                  int64_t lda, const float *B_hi, const float *B_lo, int64_t ldb, float *C_hi,
                  float *C_lo, int64_t ldc, int32_t algo, void *ws, size_t ws_bytes, void *stream)
{
    if (M < 0 || N < 0 || K < 0 || lda < K || ldb < N || ldc < N)
        return FF_ERR_SIZE;
    if (algo != FF_GEMM_FMA_LOOP && algo != FF_GEMM_SLICED_BF16 && algo != FF_GEMM_SLICED_I8)
        return FF_ERR_ARG;
    if (M == 0 || N == 0)
        return FF_OK;
    if (!C_hi || !C_lo || (K > 0 && (!A_hi || !A_lo || !B_hi || !B_lo)))
        return FF_ERR_NULL;
    for (const void *p : {static_cast<const void *>(A_hi), static_cast<const void *>(A_lo),
                          static_cast<const void *>(B_hi), static_cast<const void *>(B_lo),
                          static_cast<const void *>(C_hi), static_cast<const void *>(C_lo)})
        if (!ffh::aligned(p, 4))
            return FF_ERR_ALIGN;
    if (ffh::cdiv(M, 64) > 65535 || ffh::cdiv(N, 64) > INT32_MAX)
        return FF_ERR_SIZE;
    hipStream_t st = ffh::as_stream(stream);
    switch (algo) {
    case FF_GEMM_FMA_LOOP:
        hipLaunchKernelGGL(gemm_fma_loop,
                           dim3(static_cast<unsigned>(ffh::cdiv(N, kPT)),
                                static_cast<unsigned>(ffh::cdiv(M, kPT))),
                           dim3(256), 0, st, M, N, K, A_hi, A_lo, lda, B_hi, B_lo, ldb, C_hi, C_lo,
                           ldc);
        return ffh::launch_status();
    case FF_GEMM_SLICED_BF16:
        return sliced_gemm<DigitsBF16>(M, N, K, A_hi, A_lo, lda, B_hi, B_lo, ldb, C_hi, C_lo, ldc,
                                       ws, ws_bytes, st);
    default:
        return sliced_gemm<DigitsI8>(M, N, K, A_hi, A_lo, lda, B_hi, B_lo, ldb, C_hi, C_lo, ldc,
                                     ws, ws_bytes, st);
    }
}

} // extern "C"
