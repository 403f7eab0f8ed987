// ff_reduce.hip -- batched float-float dot products and sums.
//
// Data: vector v is [offsets[v], offsets[v+1]) of the concatenated inputs
// (binary32 x, y, or float-float planes xh, xl, yh, yl).  A vector is cut
// into chunks of `chunk` elements.  Four stream-ordered launches:
//   plan      one workgroup: chunk counts per vector and their exclusive scan
//   records   one wavefront per vector: the element range of each chunk
//   partials  persistent: each wavefront of the grid is a worker, and chunk
//             c is reduced by worker c mod (grid * waves per workgroup) into
//             a float-float partial
//   combine   one wavefront per vector: Add22 of the vector's partials
// Launch boundaries order the phases, so no fences or atomics are needed: a
// device-scope fence on gfx950 writes back and invalidates the L2 of the
// issuing XCD, which per chunk cost more than the chunk's own traffic.
//
// Per element the binary32 path reads 8 bytes and performs TwoProd (2 VALU)
// plus Add22 (~14 VALU): ~2 operations per byte, under the ~9.8 ops/byte
// ridge of gfx950 (78.6 T binary32 operations/s over 8 TB/s), so the
// partials launch is HBM-bound.  The float-float path reads 16 bytes and
// performs Mul22 + Add22 (~27 VALU) per element.
//
// Workspace layout (each section 256-byte aligned):
//   chunk_start int64[nvec + 1]  first chunk of each vector (exclusive scan)
//   ranges      int64x2[cap]     element range [s, e) of each chunk
//   partials    float2[cap]      float-float partial of each chunk
// with cap = total_len / chunk + nvec chunks at most.
#include <atomic>

#include "ff_device.h"
#include "ff_host.h"

namespace ffk {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kPlanBlock = 1024;

struct Workspace {
    int64_t *chunk_start;
    longlong2 *ranges;
    float2 *partials;
    int64_t cap;
};

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

inline int64_t chunk_capacity(int64_t total, int32_t nvec, int64_t chunk)
{
    return total / chunk + nvec;
}

inline size_t workspace_bytes(int64_t total, int32_t nvec, int64_t chunk)
{
    const int64_t cap = chunk_capacity(total, nvec, chunk);
    return align256(sizeof(int64_t) * (nvec + 1)) + align256(sizeof(longlong2) * cap) +
           align256(sizeof(float2) * cap);
}

inline Workspace carve(void *ws, int64_t total, int32_t nvec, int64_t chunk)
{
    Workspace w;
    char *p = static_cast<char *>(ws);
    w.cap = chunk_capacity(total, nvec, chunk);
    w.chunk_start = reinterpret_cast<int64_t *>(p);
    p += align256(sizeof(int64_t) * (nvec + 1));
    w.ranges = reinterpret_cast<longlong2 *>(p);
    p += align256(sizeof(longlong2) * w.cap);
    w.partials = reinterpret_cast<float2 *>(p);
    return w;
}

__device__ __forceinline__ int64_t clamp_offset(int64_t o, int64_t total)
{
    return o < 0 ? 0 : (o > total ? total : o);
}

// Planning launch (one workgroup): chunk counts of the vectors and their
// exclusive scan.  Each round covers kPlanItems consecutive vectors per
// thread: a serial scan in the thread, a shuffle scan across the wavefront,
// and a scan of the wavefront totals by the first wavefront.
constexpr int kPlanItems = 4;

__device__ __forceinline__ int64_t wave_inclusive_scan(int64_t v, int lane)
{
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int64_t o = __shfl_up(v, d, 64);
        if (lane >= d)
            v += o;
    }
    return v;
}

__global__ __launch_bounds__(kPlanBlock) void dot_plan(const int64_t *__restrict__ offsets,
                                                       int32_t nvec, int64_t total, int64_t chunk,
                                                       Workspace w)
{
    constexpr int kWaves = kPlanBlock / 64;
    __shared__ int64_t wave_sum[kWaves];
    __shared__ int64_t carry;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid == 0)
        carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < nvec; base += kPlanBlock * kPlanItems) {
        int64_t n[kPlanItems];
        int64_t mine = 0;
#pragma unroll
        for (int k = 0; k < kPlanItems; ++k) {
            const int64_t v = base + static_cast<int64_t>(tid) * kPlanItems + k;
            n[k] = 0;
            if (v < nvec) {
                const int64_t b = clamp_offset(offsets[v], total);
                const int64_t e = clamp_offset(offsets[v + 1], total);
                const int64_t len = e > b ? e - b : 0;
                n[k] = (len + chunk - 1) / chunk;
            }
            mine += n[k];
        }
        const int64_t incl = wave_inclusive_scan(mine, lane);
        if (lane == 63)
            wave_sum[wave] = incl;
        __syncthreads();
        if (wave == 0) {
            const int64_t ws = lane < kWaves ? wave_sum[lane] : 0;
            const int64_t wincl = wave_inclusive_scan(ws, lane);
            if (lane < kWaves)
                wave_sum[lane] = wincl - ws;   // exclusive
        }
        __syncthreads();
        int64_t run = carry + wave_sum[wave] + incl - mine;
#pragma unroll
        for (int k = 0; k < kPlanItems; ++k) {
            const int64_t v = base + static_cast<int64_t>(tid) * kPlanItems + k;
            if (v < nvec)
                w.chunk_start[v] = run;
            run += n[k];
        }
        __syncthreads();
        if (tid == kPlanBlock - 1)
            carry = run;   // the last thread's running total ends the round
        __syncthreads();
    }
    if (tid == 0)
        w.chunk_start[nvec] = carry;
}

// One wavefront per vector writes the element ranges of its chunks.
// Chunks beyond the workspace capacity are never recorded.
__global__ __launch_bounds__(256) void dot_ranges(const int64_t *__restrict__ offsets,
                                                  int32_t nvec, int64_t total, int64_t chunk,
                                                  Workspace w)
{
    const int64_t v = static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (v >= nvec)
        return;
    const int64_t vb = clamp_offset(offsets[v], total);
    const int64_t ve = clamp_offset(offsets[v + 1], total);
    const int64_t c0 = w.chunk_start[v];
    int64_t c1 = w.chunk_start[v + 1];
    c1 = c1 < w.cap ? c1 : w.cap;
    for (int64_t c = c0 + lane; c < c1; c += 64) {
        const int64_t rs = vb + (c - c0) * chunk;
        const int64_t re = ve < rs + chunk ? ve : rs + chunk;
        w.ranges[c] = make_longlong2(rs, re);
    }
}

// Accumulation policies.  A partial is a pair of binary32 words (h, l).
// AccFF: float-float accumulation, every term and every partial added with
// Add22 (section 4.1); the pair is the result.
struct AccFF {
    __device__ __forceinline__ static void add(float &h, float &l, float ph, float pl)
    {
        ffd::add22(h, l, ph, pl, h, l);
    }
    __device__ __forceinline__ static void merge(float &h, float &l, float oh, float ol)
    {
        ffd::add22(h, l, oh, ol, h, l);
    }
    __device__ __forceinline__ static void finish(float &, float &) {}
};
// AccComp: compensated accumulation (Sum2 / Dot2 of Ogita, Rump and Oishi,
// 2005): h is a running binary32 sum whose TwoSum rounding errors, and the
// terms' low words, are added in binary32 into l.  Two partials merge the
// same way (symmetric in its operands, so a butterfly leaves every lane with
// the same bits).  The result is Add12(h, l): its high word is the
// algorithm's rounded result h (+) l.
struct AccComp {
    __device__ __forceinline__ static void add(float &h, float &l, float ph, float pl)
    {
        float q;
        ffd::add12(h, ph, h, q);
        l = l + (q + pl);
    }
    __device__ __forceinline__ static void merge(float &h, float &l, float oh, float ol)
    {
        float q;
        ffd::add12(h, oh, h, q);
        l = (l + ol) + q;
    }
    __device__ __forceinline__ static void finish(float &h, float &l) { ffd::add12(h, l, h, l); }
};

// Butterfly all-reduce of a partial over the 64 lanes of a wavefront.
template <class Acc>
__device__ __forceinline__ void wave_allreduce(float &h, float &l)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        const float oh = __shfl_xor(h, m, 64);
        const float ol = __shfl_xor(l, m, 64);
        Acc::merge(h, l, oh, ol);
    }
}

// One wavefront per vector: the vector's chunk partials merged lane-strided
// in chunk order, then a butterfly; (0, 0) for an empty vector.
template <class Acc>
__global__ __launch_bounds__(256) void dot_combine(int32_t nvec, Workspace w,
                                                   float *__restrict__ out_hi,
                                                   float *__restrict__ out_lo)
{
    const int64_t v = static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (v >= nvec)
        return;
    const int64_t c0 = w.chunk_start[v];
    int64_t c1 = w.chunk_start[v + 1];
    c1 = c1 < w.cap ? c1 : w.cap;
    float h = 0.0f, l = 0.0f;
    for (int64_t c = c0 + lane; c < c1; c += 64) {
        const float2 p = w.partials[c];
        Acc::merge(h, l, p.x, p.y);
    }
    wave_allreduce<Acc>(h, l);
    Acc::finish(h, l);
    if (lane == 0) {
        out_hi[v] = h;
        out_lo[v] = l;
    }
}

// Input kinds.  Terms<In> loads the float4 group g (elements 4g .. 4g+3)
// of every input plane, and forms each element's exact term as a pair
// (TwoProd of binary32 inputs, Mul22 of float-float inputs, the value
// itself for sums).
struct InF32 {
    const float *x, *y;
};
struct InFF {
    const float *xh, *xl, *yh, *yl;
};
struct InSumF32 {
    const float *x;
};
struct InSumFF {
    const float *xh, *xl;
};

template <int P>
struct Planes {
    f32x4 p[P];
};

__device__ __forceinline__ f32x4 load_group(const float *a, int64_t g)
{
    return __builtin_nontemporal_load(reinterpret_cast<const f32x4 *>(a) + g);
}

template <class In>
struct Terms;

template <>
struct Terms<InF32> {
    using G = Planes<2>;
    __device__ __forceinline__ static G load(const InF32 &in, int64_t g)
    {
        return G{{load_group(in.x, g), load_group(in.y, g)}};
    }
    __device__ __forceinline__ static void term(const G &q, int k, float &ph, float &pl)
    {
        ffd::mul12_fma(q.p[0][k], q.p[1][k], ph, pl);
    }
    __device__ __forceinline__ static void one(const InF32 &in, int64_t i, float &ph, float &pl)
    {
        ffd::mul12_fma(in.x[i], in.y[i], ph, pl);
    }
};

template <>
struct Terms<InFF> {
    using G = Planes<4>;
    __device__ __forceinline__ static G load(const InFF &in, int64_t g)
    {
        return G{{load_group(in.xh, g), load_group(in.xl, g), load_group(in.yh, g),
                  load_group(in.yl, g)}};
    }
    __device__ __forceinline__ static void term(const G &q, int k, float &ph, float &pl)
    {
        ffd::mul22<false>(q.p[0][k], q.p[1][k], q.p[2][k], q.p[3][k], ph, pl);
    }
    __device__ __forceinline__ static void one(const InFF &in, int64_t i, float &ph, float &pl)
    {
        ffd::mul22<false>(in.xh[i], in.xl[i], in.yh[i], in.yl[i], ph, pl);
    }
};

template <>
struct Terms<InSumF32> {
    using G = Planes<1>;
    __device__ __forceinline__ static G load(const InSumF32 &in, int64_t g)
    {
        return G{{load_group(in.x, g)}};
    }
    // term = (x_i, 0): the binary32 value itself
    __device__ __forceinline__ static void term(const G &q, int k, float &ph, float &pl)
    {
        ph = q.p[0][k];
        pl = 0.0f;
    }
    __device__ __forceinline__ static void one(const InSumF32 &in, int64_t i, float &ph,
                                               float &pl)
    {
        ph = in.x[i];
        pl = 0.0f;
    }
};

template <>
struct Terms<InSumFF> {
    using G = Planes<2>;
    __device__ __forceinline__ static G load(const InSumFF &in, int64_t g)
    {
        return G{{load_group(in.xh, g), load_group(in.xl, g)}};
    }
    __device__ __forceinline__ static void term(const G &q, int k, float &ph, float &pl)
    {
        ph = q.p[0][k];
        pl = q.p[1][k];
    }
    __device__ __forceinline__ static void one(const InSumFF &in, int64_t i, float &ph,
                                               float &pl)
    {
        ph = in.xh[i];
        pl = in.xl[i];
    }
};

template <class In, class Acc>
__device__ __forceinline__ void add_group(const typename Terms<In>::G &q, float2 acc[4])
{
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        float ph, pl;
        Terms<In>::term(q, k, ph, pl);
        Acc::add(acc[k].x, acc[k].y, ph, pl);
    }
}

// The persistent partials launch.  Each wavefront is an independent worker:
// global wavefront w reduces chunks w, w + W, w + 2W, ... (W wavefronts in
// the grid) to a partial with a butterfly, no barriers.
// VEC (all planes 16-byte aligned): the float4 groups lying wholly inside
// the chunk are read UNROLL at a time per lane, all loads issued before any
// arithmetic; the at most 3 + 3 elements before the first and after the
// last whole group are read one by one.  Otherwise every element is read
// on its own.
template <class In, class Acc, int BLOCK, int UNROLL, bool VEC>
__global__ __launch_bounds__(BLOCK) void dot_partials(In in, Workspace w, int32_t nvec)
{
    constexpr int kWaves = BLOCK / 64;
    const int lane = threadIdx.x & 63;
    const int64_t gw = static_cast<int64_t>(blockIdx.x) * kWaves + (threadIdx.x >> 6);
    const int64_t nw = static_cast<int64_t>(gridDim.x) * kWaves;
    int64_t nchunks = w.chunk_start[nvec];
    if (nchunks > w.cap)
        nchunks = w.cap;

    for (int64_t c = gw; c < nchunks; c += nw) {
        const longlong2 r = w.ranges[c];
        const int64_t s = r.x, e = r.y;

        float2 acc[4];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            acc[k] = make_float2(0.0f, 0.0f);
        if (VEC) {
            const int64_t ga = (s + 3) >> 2;   // first whole group
            int64_t gb = e >> 2;               // end of the whole groups
            if (gb < ga)
                gb = ga;                       // s and e inside one group
            int64_t g = ga + lane;
            for (; g + (UNROLL - 1) * 64 < gb; g += 64 * UNROLL) {
                typename Terms<In>::G q[UNROLL];
#pragma unroll
                for (int u = 0; u < UNROLL; ++u)
                    q[u] = Terms<In>::load(in, g + u * 64);
#pragma unroll
                for (int u = 0; u < UNROLL; ++u)
                    add_group<In, Acc>(q[u], acc);
            }
            for (; g < gb; g += 64)
                add_group<In, Acc>(Terms<In>::load(in, g), acc);
            // head [s, 4 ga) and tail [4 gb, e) elements, by lanes 0..2 and
            // 32..34 (when a chunk lies inside one group, gb = ga and the
            // head covers it)
            const int64_t head_end = 4 * ga < e ? 4 * ga : e;
            const int64_t tail_beg = 4 * gb > s ? 4 * gb : s;
            int64_t i = -1;
            if (lane < 3 && s + lane < head_end)
                i = s + lane;
            else if (lane >= 32 && lane < 35 && tail_beg + (lane - 32) < e)
                i = tail_beg + (lane - 32);
            if (i >= 0) {
                float ph, pl;
                Terms<In>::one(in, i, ph, pl);
                Acc::add(acc[0].x, acc[0].y, ph, pl);
            }
        } else {
            for (int64_t i = s + lane; i < e; i += 64) {
                float ph, pl;
                Terms<In>::one(in, i, ph, pl);
                Acc::add(acc[0].x, acc[0].y, ph, pl);
            }
        }
        float h = acc[0].x, l = acc[0].y;
        Acc::merge(h, l, acc[1].x, acc[1].y);
        float h2 = acc[2].x, l2 = acc[2].y;
        Acc::merge(h2, l2, acc[3].x, acc[3].y);
        Acc::merge(h, l, h2, l2);
        wave_allreduce<Acc>(h, l);
        if (lane == 0)
            w.partials[c] = make_float2(h, l);
    }
}

struct Cfg {
    int block, unroll, grid;
    int64_t chunk;
};

ff_status resolve_cfg(const ff_dot_cfg *cfg, Cfg &out)
{
    // defaults: the fastest shape on 4096 vectors of 2^6 .. 2^20 elements
    out.block = 512;
    out.chunk = 16384;
    out.grid = 0;
    out.unroll = 8;
    if (cfg) {
        if (cfg->block)
            out.block = cfg->block;
        if (cfg->chunk)
            out.chunk = cfg->chunk;
        if (cfg->grid)
            out.grid = cfg->grid;
        if (cfg->unroll)
            out.unroll = cfg->unroll;
    }
    if (out.block != 256 && out.block != 512)
        return FF_ERR_ARG;
    if (out.unroll != 1 && out.unroll != 2 && out.unroll != 4 && out.unroll != 8)
        return FF_ERR_ARG;
    if (out.chunk < 64 || out.chunk % 4 != 0)
        return FF_ERR_ARG;
    if (out.grid < 0)
        return FF_ERR_ARG;
    return FF_OK;
}

int default_grid()
{
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        cus = 256;  // MI355X's count when the query fails
    return 8 * (cus > 0 ? cus : 256);
}

template <class In, class Acc, int BLOCK, int UNROLL>
void launch_partials(bool vec, int grid, hipStream_t st, const In &in, const Workspace &w,
                     int32_t nvec)
{
    if (vec)
        hipLaunchKernelGGL((dot_partials<In, Acc, BLOCK, UNROLL, true>), dim3(grid), dim3(BLOCK),
                           0, st, in, w, nvec);
    else
        hipLaunchKernelGGL((dot_partials<In, Acc, BLOCK, 1, false>), dim3(grid), dim3(BLOCK), 0,
                           st, in, w, nvec);
}

template <class In, class Acc = AccFF>
ff_status dot_batched_entry(const In &in, bool vec, const int64_t *offsets, int32_t nvec,
                            int64_t total, const ff_dot_cfg *cfg_in, void *ws, size_t ws_bytes,
                            float *out_hi, float *out_lo, void *stream_ptr)
{
    Cfg cfg;
    const ff_status cs = resolve_cfg(cfg_in, cfg);
    if (cs != FF_OK)
        return cs;
    if (nvec == 0)
        return FF_OK;
    if (!offsets || !out_hi || !out_lo || !ws)
        return FF_ERR_NULL;
    if (!ffh::aligned(offsets, 8) || !ffh::aligned(out_hi, 4) || !ffh::aligned(out_lo, 4) ||
        !ffh::aligned(ws, 256))
        return FF_ERR_ALIGN;
    if (ws_bytes < workspace_bytes(total, nvec, cfg.chunk))
        return FF_ERR_WORKSPACE;
    hipStream_t st = ffh::as_stream(stream_ptr);
    const Workspace w = carve(ws, total, nvec, cfg.chunk);
    const int grid = cfg.grid ? cfg.grid : default_grid();
    const unsigned wave_blocks = static_cast<unsigned>(ffh::cdiv(nvec, 4));
    hipLaunchKernelGGL(dot_plan, dim3(1), dim3(kPlanBlock), 0, st, offsets, nvec, total,
                       cfg.chunk, w);
    hipLaunchKernelGGL(dot_ranges, dim3(wave_blocks), dim3(256), 0, st, offsets, nvec, total,
                       cfg.chunk, w);
#define FF_DOT_LAUNCH(B, U) launch_partials<In, Acc, B, U>(vec, grid, st, in, w, nvec)
    if (cfg.block == 256) {
        switch (cfg.unroll) {
        case 1: FF_DOT_LAUNCH(256, 1); break;
        case 2: FF_DOT_LAUNCH(256, 2); break;
        case 4: FF_DOT_LAUNCH(256, 4); break;
        default: FF_DOT_LAUNCH(256, 8); break;
        }
    } else {
        switch (cfg.unroll) {
        case 1: FF_DOT_LAUNCH(512, 1); break;
        case 2: FF_DOT_LAUNCH(512, 2); break;
        case 4: FF_DOT_LAUNCH(512, 4); break;
        default: FF_DOT_LAUNCH(512, 8); break;
        }
    }
#undef FF_DOT_LAUNCH
    hipLaunchKernelGGL(dot_combine<Acc>, dim3(wave_blocks), dim3(256), 0, st, nvec, w, out_hi,
                       out_lo);
    return ffh::launch_status();
}

} // namespace ffk

using namespace ffk;

extern "C" {

size_t ff_dot_batched_workspace_size(int64_t total_len, int32_t nvec, const ff_dot_cfg *cfg)
{
    Cfg c;
    if (total_len < 0 || nvec < 0 || resolve_cfg(cfg, c) != FF_OK)
        return 0;
    return workspace_bytes(total_len, nvec, c.chunk);
}

ff_status ff_dot_batched(const float *x, const float *y, const int64_t *offsets, int32_t nvec,
                         int64_t total_len, const ff_dot_cfg *cfg, void *ws, size_t ws_bytes,
                         float *out_hi, float *out_lo, void *stream)
{
    if (nvec < 0 || total_len < 0)
        return FF_ERR_SIZE;
    if (total_len > 0 && (!x || !y))
        return FF_ERR_NULL;
    if (!ffh::aligned(x, 4) || !ffh::aligned(y, 4))
        return FF_ERR_ALIGN;
    const bool vec = ffh::aligned(x, 16) && ffh::aligned(y, 16);
    return dot_batched_entry(InF32{x, y}, vec, offsets, nvec, total_len, cfg, ws, ws_bytes,
                             out_hi, out_lo, stream);
}

ff_status ff_dot_ff_batched(const float *x_hi, const float *x_lo, const float *y_hi,
                            const float *y_lo, const int64_t *offsets, int32_t nvec,
                            int64_t total_len, const ff_dot_cfg *cfg, void *ws, size_t ws_bytes,
                            float *out_hi, float *out_lo, void *stream)
{
    if (nvec < 0 || total_len < 0)
        return FF_ERR_SIZE;
    if (total_len > 0 && (!x_hi || !x_lo || !y_hi || !y_lo))
        return FF_ERR_NULL;
    const void *planes[4] = {x_hi, x_lo, y_hi, y_lo};
    bool vec = true;
    for (const void *p : planes) {
        if (!ffh::aligned(p, 4))
            return FF_ERR_ALIGN;
        vec = vec && ffh::aligned(p, 16);
    }
    return dot_batched_entry(InFF{x_hi, x_lo, y_hi, y_lo}, vec, offsets, nvec, total_len, cfg, ws,
                             ws_bytes, out_hi, out_lo, stream);
}

ff_status ff_sum_batched(const float *x, const int64_t *offsets, int32_t nvec, int64_t total_len,
                         const ff_dot_cfg *cfg, void *ws, size_t ws_bytes, float *out_hi,
                         float *out_lo, void *stream)
{
    if (nvec < 0 || total_len < 0)
        return FF_ERR_SIZE;
    if (total_len > 0 && !x)
        return FF_ERR_NULL;
    if (!ffh::aligned(x, 4))
        return FF_ERR_ALIGN;
    return dot_batched_entry(InSumF32{x}, ffh::aligned(x, 16), offsets, nvec, total_len, cfg, ws,
                             ws_bytes, out_hi, out_lo, stream);
}

ff_status ff_sum_ff_batched(const float *x_hi, const float *x_lo, const int64_t *offsets,
                            int32_t nvec, int64_t total_len, const ff_dot_cfg *cfg, void *ws,
                            size_t ws_bytes, float *out_hi, float *out_lo, void *stream)
{
    if (nvec < 0 || total_len < 0)
        return FF_ERR_SIZE;
    if (total_len > 0 && (!x_hi || !x_lo))
        return FF_ERR_NULL;
    if (!ffh::aligned(x_hi, 4) || !ffh::aligned(x_lo, 4))
        return FF_ERR_ALIGN;
    const bool vec = ffh::aligned(x_hi, 16) && ffh::aligned(x_lo, 16);
    return dot_batched_entry(InSumFF{x_hi, x_lo}, vec, offsets, nvec, total_len, cfg, ws, ws_bytes,
                             out_hi, out_lo, stream);
}

ff_status ff_dot2_batched(const float *x, const float *y, const int64_t *offsets, int32_t nvec,
                          int64_t total_len, const ff_dot_cfg *cfg, void *ws, size_t ws_bytes,
                          float *out_hi, float *out_lo, void *stream)
{
    if (nvec < 0 || total_len < 0)
        return FF_ERR_SIZE;
    if (total_len > 0 && (!x || !y))
        return FF_ERR_NULL;
    if (!ffh::aligned(x, 4) || !ffh::aligned(y, 4))
        return FF_ERR_ALIGN;
    const bool vec = ffh::aligned(x, 16) && ffh::aligned(y, 16);
    return dot_batched_entry<InF32, AccComp>(InF32{x, y}, vec, offsets, nvec, total_len, cfg, ws,
                                             ws_bytes, out_hi, out_lo, stream);
}

ff_status ff_sum2_batched(const float *x, const int64_t *offsets, int32_t nvec,
                          int64_t total_len, const ff_dot_cfg *cfg, void *ws, size_t ws_bytes,
                          float *out_hi, float *out_lo, void *stream)
{
    if (nvec < 0 || total_len < 0)
        return FF_ERR_SIZE;
    if (total_len > 0 && !x)
        return FF_ERR_NULL;
    if (!ffh::aligned(x, 4))
        return FF_ERR_ALIGN;
    return dot_batched_entry<InSumF32, AccComp>(InSumF32{x}, ffh::aligned(x, 16), offsets, nvec,
                                                total_len, cfg, ws, ws_bytes, out_hi, out_lo,
                                                stream);
}

} // extern "C"

namespace {

// Scratch memory of the allocation-free batched dot: a static device array,
// one copy per device the library runs on, held until the process ends.
// Host code never passes the array's name to a kernel (on the host it is
// only a stand-in for the symbol): the device address is looked up once per
// device with hipGetSymbolAddress and kept in `g_scratch_addr`.
static __device__ __align__(256) unsigned char scratch[FF_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxScratchDevices = 64;
std::atomic<void *> g_scratch_addr[kMaxScratchDevices];

// Device address of `scratch` on the current device (looked up on the
// first call on that device; a concurrent first call stores the same value).
ff_status scratch_on_current_device(void **addr)
{
    int dev = 0;
    hipError_t err = hipGetDevice(&dev);
    if (err != hipSuccess)
        return ffh::hip_failure(err);
    if (dev < 0 || dev >= kMaxScratchDevices)
        return FF_ERR_UNSUPPORTED;
    void *p = g_scratch_addr[dev].load(std::memory_order_acquire);
    if (!p) {
        err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (err != hipSuccess)
            return ffh::hip_failure(err);
        if (!p)
            return FF_ERR_HIP;
        g_scratch_addr[dev].store(p, std::memory_order_release);
    }
    *addr = p;
    return FF_OK;
}

} // namespace

extern "C" {

ff_status ff_dot_batched_noalloc(const float *x, const float *y, const int64_t *offsets,
                                 int32_t nvec, int64_t total_len, const ff_dot_cfg *cfg,
                                 float *out_hi, float *out_lo, void *stream)
{
    // the argument checks of ff_dot_batched, in its order, plus the scratch
    // limit, all before any HIP call
    if (nvec < 0 || total_len < 0)
        return FF_ERR_SIZE;
    if (total_len > 0 && (!x || !y))
        return FF_ERR_NULL;
    if (!ffh::aligned(x, 4) || !ffh::aligned(y, 4))
        return FF_ERR_ALIGN;
    Cfg c;
    const ff_status cs = resolve_cfg(cfg, c);
    if (cs != FF_OK)
        return cs;
    if (nvec == 0)
        return FF_OK;
    if (!offsets || !out_hi || !out_lo)
        return FF_ERR_NULL;
    if (!ffh::aligned(offsets, 8) || !ffh::aligned(out_hi, 4) || !ffh::aligned(out_lo, 4))
        return FF_ERR_ALIGN;
    if (workspace_bytes(total_len, nvec, c.chunk) > FF_NOALLOC_SCRATCH_BYTES)
        return FF_ERR_WORKSPACE;
    void *ws = nullptr;
    const ff_status ss = scratch_on_current_device(&ws);
    if (ss != FF_OK)
        return ss;
    const bool vec = ffh::aligned(x, 16) && ffh::aligned(y, 16);
    return dot_batched_entry(InF32{x, y}, vec, offsets, nvec, total_len, cfg, ws,
                             FF_NOALLOC_SCRATCH_BYTES, out_hi, out_lo, stream);
}

ff_status ff_dot_batched_autotune(const float *x, const float *y, const int64_t *offsets,
                                  int32_t nvec, int64_t total_len, void *ws, size_t ws_bytes,
                                  float *out_hi, float *out_lo, int32_t reps, void *stream,
                                  ff_dot_cfg *best, float *best_ms)
{
    if (!best || !best_ms)
        return FF_ERR_NULL;
    if (reps < 1)
        return FF_ERR_ARG;
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return ffh::hip_failure(hipGetLastError());
    static const int kBlocks[] = {256, 512};
    static const int kUnrolls[] = {1, 2, 4, 8};
    static const int kChunks[] = {1024, 2048, 4096, 8192, 16384, 32768};
    static const int kPerCu[] = {2, 4, 8, 16};
    hipStream_t st = ffh::as_stream(stream);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess)
        return ffh::hip_failure(hipGetLastError());
    if (hipEventCreate(&e1) != hipSuccess) {
        const ff_status failed = ffh::hip_failure(hipGetLastError());
        (void)hipEventDestroy(e0);
        return failed;
    }
    ff_status status = FF_OK;
    float best_time = -1.0f;
    for (int blk : kBlocks)
        for (int un : kUnrolls)
            for (int ch : kChunks)
                for (int pc : kPerCu) {
                    ff_dot_cfg c{blk, ch, pc * cus, un};
                    if (ff_dot_batched_workspace_size(total_len, nvec, &c) > ws_bytes)
                        continue;
                    // one untimed launch, then reps timed launches
                    status = ff_dot_batched(x, y, offsets, nvec, total_len, &c, ws, ws_bytes,
                                            out_hi, out_lo, stream);
                    if (status != FF_OK)
                        goto done;
                    if (hipEventRecord(e0, st) != hipSuccess) {
                        status = ffh::hip_failure(hipGetLastError());
                        goto done;
                    }
                    for (int r = 0; r < reps && status == FF_OK; ++r)
                        status = ff_dot_batched(x, y, offsets, nvec, total_len, &c, ws, ws_bytes,
                                                out_hi, out_lo, stream);
                    if (status != FF_OK)
                        goto done;
                    float ms = 0.0f;
                    if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                        hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                        status = ffh::hip_failure(hipGetLastError());
                        goto done;
                    }
                    ms /= reps;
                    if (best_time < 0.0f || ms < best_time) {
                        best_time = ms;
                        *best = c;
                    }
                }
    if (best_time < 0.0f)
        status = FF_ERR_WORKSPACE;
    *best_ms = best_time;
done:
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return status;
}

} // extern "C"
