// ff_reduce.hip -- batched float-float dot products and sums.
//
// Data: vector v is [offsets[v], offsets[v+1]) of the concatenated inputs
// (binary32 x, y, or float-float planes xh, xl, yh, yl).  A vector is cut
// into chunks of `chunk` = block * unroll elements.  Four stream-ordered
// launches:
//   plan      one workgroup: chunk counts per vector and their exclusive scan
//   records   one wavefront per vector: the element range of each chunk
//   partials  one workgroup per chunk, launched in chunk order (which is
//             memory order): thread t takes the chunk's elements t + block k
//             (k < unroll) of every plane with 4-byte loads, all issued
//             before any arithmetic, accumulates them in order, and the
//             workgroup reduces its threads to the chunk's float-float partial
//   combine   one wavefront per vector: Add22 of the vector's partials
// The resident workgroups of the partials launch sweep memory together, the
// pattern the HBM streams fastest (the elementwise operators' lesson): on
// the 4096-vector batch it moved 0.79-0.85 of the HBM peak for all four input
// kinds and any placement of the planes, where persistent workers reducing
// chunks spread over memory had reached 0.80 for binary32 dots but 0.60-0.75
// for float-float inputs and sums.  Launch boundaries order the phases, so no
// fences or atomics are needed: a device-scope fence on gfx950 writes back and
// invalidates the L2 of the issuing XCD.
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

// Input kinds.  Terms<In>::load reads element i of every input plane (one
// 4-byte load each) and Terms<In>::term forms the element's exact term as a
// pair: TwoProd of binary32 inputs, Mul22 of float-float inputs, the value
// itself for sums.
struct InF32 {
    const float *x, *y;
    static constexpr int kPlanes = 2;
};
struct InFF {
    const float *xh, *xl, *yh, *yl;
    static constexpr int kPlanes = 4;
};
struct InSumF32 {
    const float *x;
    static constexpr int kPlanes = 1;
};
struct InSumFF {
    const float *xh, *xl;
    static constexpr int kPlanes = 2;
};

__device__ __forceinline__ float load_nt(const float *p, int64_t i)
{
    return __builtin_nontemporal_load(p + i);
}

template <class In>
struct Terms;

template <>
struct Terms<InF32> {
    __device__ __forceinline__ static void load(const InF32 &in, int64_t i, float *v)
    {
        v[0] = load_nt(in.x, i);
        v[1] = load_nt(in.y, i);
    }
    __device__ __forceinline__ static void term(const float *v, float &ph, float &pl)
    {
        ffd::mul12_fma(v[0], v[1], ph, pl);
    }
};

template <>
struct Terms<InFF> {
    __device__ __forceinline__ static void load(const InFF &in, int64_t i, float *v)
    {
        v[0] = load_nt(in.xh, i);
        v[1] = load_nt(in.xl, i);
        v[2] = load_nt(in.yh, i);
        v[3] = load_nt(in.yl, i);
    }
    __device__ __forceinline__ static void term(const float *v, float &ph, float &pl)
    {
        ffd::mul22<false>(v[0], v[1], v[2], v[3], ph, pl);
    }
};

template <>
struct Terms<InSumF32> {
    __device__ __forceinline__ static void load(const InSumF32 &in, int64_t i, float *v)
    {
        v[0] = load_nt(in.x, i);
    }
    // term = (x_i, 0): the binary32 value itself
    __device__ __forceinline__ static void term(const float *v, float &ph, float &pl)
    {
        ph = v[0];
        pl = 0.0f;
    }
};

template <>
struct Terms<InSumFF> {
    __device__ __forceinline__ static void load(const InSumFF &in, int64_t i, float *v)
    {
        v[0] = load_nt(in.xh, i);
        v[1] = load_nt(in.xl, i);
    }
    __device__ __forceinline__ static void term(const float *v, float &ph, float &pl)
    {
        ph = v[0];
        pl = v[1];
    }
};

// The partials launch: workgroup c reduces chunk c (c < the chunk count;
// the grid holds the capacity, and the workgroups past the count return).
// Thread t loads the chunk's elements s + t + BLOCK k, k < PER, of every
// plane (each wavefront load is 256 contiguous bytes of a plane; any 4-byte
// alignment), then adds their terms in k order into one float-float
// accumulator.  A butterfly over the wavefront, then the wavefronts' sums in
// index order, give the chunk's partial.  The order is fixed by (BLOCK,
// PER), so results are reproducible run to run.
template <class In, class Acc, int BLOCK, int PER>
__global__ __launch_bounds__(BLOCK) void dot_chunks(In in, Workspace w, int32_t nvec)
{
    constexpr int kWaves = BLOCK / 64;
    __shared__ float2 wave_part[kWaves];
    const int64_t c = blockIdx.x;
    int64_t nchunks = w.chunk_start[nvec];
    if (nchunks > w.cap)
        nchunks = w.cap;
    if (c >= nchunks)
        return;
    const longlong2 r = w.ranges[c];
    const int64_t s = r.x, e = r.y;   // s < e: recorded chunks are not empty
    const int t = threadIdx.x;
    float v[PER][In::kPlanes];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int64_t i = s + t + static_cast<int64_t>(BLOCK) * k;
        Terms<In>::load(in, i < e ? i : s, v[k]);   // past the end: a harmless in-range load
    }
    float h = 0.0f, l = 0.0f;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int64_t i = s + t + static_cast<int64_t>(BLOCK) * k;
        if (i < e) {
            float ph, pl;
            Terms<In>::term(v[k], ph, pl);
            Acc::add(h, l, ph, pl);
        }
    }
    wave_allreduce<Acc>(h, l);
    if ((t & 63) == 0)
        wave_part[t >> 6] = make_float2(h, l);
    __syncthreads();
    if (t == 0) {
        float ph = wave_part[0].x, pl = wave_part[0].y;
#pragma unroll
        for (int q = 1; q < kWaves; ++q)
            Acc::merge(ph, pl, wave_part[q].x, wave_part[q].y);
        w.partials[c] = make_float2(ph, pl);
    }
}

struct Cfg {
    int block, unroll;
    int64_t chunk;
};

// Default launch shape, the fastest measured on MI355X for every input kind
// on the 4096-vector batch (438.9 M elements): 256 threads by 32 elements
// (chunks of 8192), 0.84 of the HBM peak for both dots and the float-float
// sum and 0.80 for the binary32 sum, against 0.75-0.83 at 128-512 threads by
// 4-16 elements.
template <class In> struct DefaultShape {
    static constexpr int kBlock = 256, kUnroll = 32;
};

bool valid_unroll(int u)
{
    return u == 1 || u == 2 || u == 4 || u == 8 || u == 16 || u == 32;
}

// A shape: block in {64, 128, 256, 512}, unroll in {1, ..., 32} (powers of
// two), chunk = block * unroll; zero fields take the kind's default (an
// unroll of zero with a chunk given takes chunk / block); grid is reserved
// and must be zero.
ff_status resolve_cfg(const ff_dot_cfg *cfg, int def_block, int def_unroll, Cfg &out)
{
    out.block = def_block;
    out.unroll = def_unroll;
    int64_t chunk = 0;
    if (cfg) {
        if (cfg->grid != 0 || cfg->block < 0 || cfg->chunk < 0 || cfg->unroll < 0)
            return FF_ERR_ARG;
        if (cfg->block)
            out.block = cfg->block;
        chunk = cfg->chunk;
        if (cfg->unroll)
            out.unroll = cfg->unroll;
        else if (chunk)
            out.unroll = chunk % out.block == 0 ? static_cast<int>(chunk / out.block) : 0;
    }
    if (out.block != 64 && out.block != 128 && out.block != 256 && out.block != 512)
        return FF_ERR_ARG;
    if (!valid_unroll(out.unroll))
        return FF_ERR_ARG;
    out.chunk = static_cast<int64_t>(out.block) * out.unroll;
    if (chunk && chunk != out.chunk)
        return FF_ERR_ARG;
    return FF_OK;
}

template <class In, class Acc, int BLOCK>
void launch_chunks(int unroll, unsigned grid, hipStream_t st, const In &in, const Workspace &w,
                   int32_t nvec)
{
    switch (unroll) {
    case 1: hipLaunchKernelGGL((dot_chunks<In, Acc, BLOCK, 1>), dim3(grid), dim3(BLOCK), 0, st, in, w, nvec); break;
    case 2: hipLaunchKernelGGL((dot_chunks<In, Acc, BLOCK, 2>), dim3(grid), dim3(BLOCK), 0, st, in, w, nvec); break;
    case 4: hipLaunchKernelGGL((dot_chunks<In, Acc, BLOCK, 4>), dim3(grid), dim3(BLOCK), 0, st, in, w, nvec); break;
    case 8: hipLaunchKernelGGL((dot_chunks<In, Acc, BLOCK, 8>), dim3(grid), dim3(BLOCK), 0, st, in, w, nvec); break;
    case 16: hipLaunchKernelGGL((dot_chunks<In, Acc, BLOCK, 16>), dim3(grid), dim3(BLOCK), 0, st, in, w, nvec); break;
    default: hipLaunchKernelGGL((dot_chunks<In, Acc, BLOCK, 32>), dim3(grid), dim3(BLOCK), 0, st, in, w, nvec); break;
    }
}

template <class In, class Acc = AccFF>
ff_status dot_batched_entry(const In &in, const int64_t *offsets, int32_t nvec, int64_t total,
                            const ff_dot_cfg *cfg_in, void *ws, size_t ws_bytes, float *out_hi,
                            float *out_lo, void *stream_ptr)
{
    Cfg cfg;
    const ff_status cs =
        resolve_cfg(cfg_in, DefaultShape<In>::kBlock, DefaultShape<In>::kUnroll, cfg);
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
    const Workspace w = carve(ws, total, nvec, cfg.chunk);
    if (w.cap > INT32_MAX)
        return FF_ERR_SIZE;
    hipStream_t st = ffh::as_stream(stream_ptr);
    const unsigned wave_blocks = static_cast<unsigned>(ffh::cdiv(nvec, 4));
    const unsigned grid = static_cast<unsigned>(w.cap);
    hipLaunchKernelGGL(dot_plan, dim3(1), dim3(kPlanBlock), 0, st, offsets, nvec, total,
                       cfg.chunk, w);
    hipLaunchKernelGGL(dot_ranges, dim3(wave_blocks), dim3(256), 0, st, offsets, nvec, total,
                       cfg.chunk, w);
    switch (cfg.block) {
    case 64: launch_chunks<In, Acc, 64>(cfg.unroll, grid, st, in, w, nvec); break;
    case 128: launch_chunks<In, Acc, 128>(cfg.unroll, grid, st, in, w, nvec); break;
    case 256: launch_chunks<In, Acc, 256>(cfg.unroll, grid, st, in, w, nvec); break;
    default: launch_chunks<In, Acc, 512>(cfg.unroll, grid, st, in, w, nvec); break;
    }
    hipLaunchKernelGGL(dot_combine<Acc>, dim3(wave_blocks), dim3(256), 0, st, nvec, w, out_hi,
                       out_lo);
    return ffh::launch_status();
}

// The smallest default chunk over the input kinds: a workspace sized for it
// serves every kind's default shape.
constexpr int64_t kSmallestDefaultChunk =
    static_cast<int64_t>(DefaultShape<InFF>::kBlock) * DefaultShape<InFF>::kUnroll;

} // namespace ffk

using namespace ffk;

extern "C" {

size_t ff_dot_batched_workspace_size(int64_t total_len, int32_t nvec, const ff_dot_cfg *cfg)
{
    // resolved with the smallest default chunk of the input kinds: enough for
    // every entry point called with this cfg
    Cfg c;
    if (total_len < 0 || nvec < 0 ||
        resolve_cfg(cfg, DefaultShape<InFF>::kBlock, DefaultShape<InFF>::kUnroll, c) != FF_OK)
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
    return dot_batched_entry(InF32{x, y}, offsets, nvec, total_len, cfg, ws, ws_bytes, out_hi,
                             out_lo, stream);
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
    for (const void *p : planes)
        if (!ffh::aligned(p, 4))
            return FF_ERR_ALIGN;
    return dot_batched_entry(InFF{x_hi, x_lo, y_hi, y_lo}, offsets, nvec, total_len, cfg, ws,
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
    return dot_batched_entry(InSumF32{x}, offsets, nvec, total_len, cfg, ws, ws_bytes, out_hi,
                             out_lo, stream);
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
    return dot_batched_entry(InSumFF{x_hi, x_lo}, offsets, nvec, total_len, cfg, ws, ws_bytes,
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
    return dot_batched_entry<InF32, AccComp>(InF32{x, y}, offsets, nvec, total_len, cfg, ws,
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
    return dot_batched_entry<InSumF32, AccComp>(InSumF32{x}, offsets, nvec, total_len, cfg, ws,
                                                ws_bytes, out_hi, out_lo, stream);
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
    const ff_status cs =
        resolve_cfg(cfg, DefaultShape<InF32>::kBlock, DefaultShape<InF32>::kUnroll, c);
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
    return dot_batched_entry(InF32{x, y}, offsets, nvec, total_len, cfg, ws,
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
    static const int kBlocks[] = {64, 128, 256, 512};
    static const int kUnrolls[] = {4, 8, 16, 32};
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
        for (int un : kUnrolls) {
            ff_dot_cfg c{blk, blk * un, 0, un};
            if (ff_dot_batched_workspace_size(total_len, nvec, &c) > ws_bytes)
                continue;
            // one untimed launch, then reps timed launches
            status = ff_dot_batched(x, y, offsets, nvec, total_len, &c, ws, ws_bytes, out_hi,
                                    out_lo, stream);
            if (status != FF_OK)
                goto done;
            if (hipEventRecord(e0, st) != hipSuccess) {
                status = ffh::hip_failure(hipGetLastError());
                goto done;
            }
            for (int r = 0; r < reps && status == FF_OK; ++r)
                status = ff_dot_batched(x, y, offsets, nvec, total_len, &c, ws, ws_bytes, out_hi,
                                        out_lo, stream);
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
