// ff_reduce.hip -- batched float-float dot products in one persistent launch.
//
// Data: vector v is [offsets[v], offsets[v+1]) of the concatenated inputs
// (binary32 x, y, or float-float planes xh, xl, yh, yl).  A vector is cut
// into chunks of `chunk` elements; chunk c of the whole batch is reduced by
// one workgroup into a float-float partial in the workspace, and the
// workgroup that finishes a vector's last chunk (completion counter per
// vector) combines that vector's partials.
//
// Per element the binary32 path reads 8 bytes and performs TwoProd (2 VALU)
// plus Add22 (~14 VALU): ~2 operations per byte, under the ~4.9 ops/byte
// ridge of gfx950 (39.3 T lane-ops/s unpacked FP32 over 8 TB/s), so the
// kernel is HBM-bound.  The float-float path reads 16 bytes and performs
// Mul22 + Add22 (~27 VALU) per element.
//
// Workspace layout (each section 256-byte aligned):
//   chunk_start int64[nvec + 1]  first chunk of each vector (exclusive scan)
//   chunk_vec   int32[cap]       owning vector of each chunk
//   counters    uint32[nvec]     chunks of the vector finished so far
//   partials    float2[cap]      float-float partial of each chunk
// with cap = total_len / chunk + nvec chunks at most.
#include "ff_device.h"
#include "ff_host.h"

namespace ffk {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kPlanBlock = 1024;

struct Workspace {
    int64_t *chunk_start;
    int32_t *chunk_vec;
    uint32_t *counters;
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
    return align256(sizeof(int64_t) * (nvec + 1)) + align256(sizeof(int32_t) * cap) +
           align256(sizeof(uint32_t) * nvec) + align256(sizeof(float2) * cap);
}

inline Workspace carve(void *ws, int64_t total, int32_t nvec, int64_t chunk)
{
    Workspace w;
    char *p = static_cast<char *>(ws);
    w.cap = chunk_capacity(total, nvec, chunk);
    w.chunk_start = reinterpret_cast<int64_t *>(p);
    p += align256(sizeof(int64_t) * (nvec + 1));
    w.chunk_vec = reinterpret_cast<int32_t *>(p);
    p += align256(sizeof(int32_t) * w.cap);
    w.counters = reinterpret_cast<uint32_t *>(p);
    p += align256(sizeof(uint32_t) * nvec);
    w.partials = reinterpret_cast<float2 *>(p);
    return w;
}

__device__ __forceinline__ int64_t clamp_offset(int64_t o, int64_t total)
{
    return o < 0 ? 0 : (o > total ? total : o);
}

// Planning launch (one workgroup): chunk counts, their exclusive scan,
// the chunk -> vector map, zeroed completion counters, and (0, 0) for empty
// vectors.  Chunks beyond the workspace capacity are never mapped.
__global__ __launch_bounds__(kPlanBlock) void dot_plan(const int64_t *__restrict__ offsets,
                                                       int32_t nvec, int64_t total, int64_t chunk,
                                                       Workspace w, float *__restrict__ out_hi,
                                                       float *__restrict__ out_lo)
{
    __shared__ int64_t scan[kPlanBlock];
    __shared__ int64_t carry;
    const int tid = threadIdx.x;
    if (tid == 0)
        carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < nvec; base += kPlanBlock) {
        const int64_t v = base + tid;
        int64_t n = 0;
        if (v < nvec) {
            const int64_t b = clamp_offset(offsets[v], total);
            const int64_t e = clamp_offset(offsets[v + 1], total);
            const int64_t len = e > b ? e - b : 0;
            n = (len + chunk - 1) / chunk;
            w.counters[v] = 0u;
            if (len == 0) {
                out_hi[v] = 0.0f;
                out_lo[v] = 0.0f;
            }
        }
        scan[tid] = n;
        __syncthreads();
        for (int d = 1; d < kPlanBlock; d <<= 1) {   // Hillis-Steele inclusive scan
            const int64_t add = tid >= d ? scan[tid - d] : 0;
            __syncthreads();
            scan[tid] += add;
            __syncthreads();
        }
        if (v < nvec)
            w.chunk_start[v] = carry + scan[tid] - n;
        __syncthreads();
        if (tid == kPlanBlock - 1)
            carry += scan[tid];
        __syncthreads();
    }
    if (tid == 0)
        w.chunk_start[nvec] = carry;
    __syncthreads();
    for (int64_t v = tid; v < nvec; v += kPlanBlock) {
        const int64_t c1 = w.chunk_start[v + 1] < w.cap ? w.chunk_start[v + 1] : w.cap;
        for (int64_t c = w.chunk_start[v]; c < c1; ++c)
            w.chunk_vec[c] = static_cast<int32_t>(v);
    }
}

// Input kinds.  load4() returns the four terms of the float4 group starting
// at element 4*g as exact float-float products; lanes outside [s, e) give 0.
struct InF32 {
    const float *x, *y;
    static constexpr int kBytes = 8;
};
struct InFF {
    const float *xh, *xl, *yh, *yl;
    static constexpr int kBytes = 16;
};
struct InSumF32 {
    const float *x;
    static constexpr int kBytes = 4;
};
struct InSumFF {
    const float *xh, *xl;
    static constexpr int kBytes = 8;
};

__device__ __forceinline__ void accumulate_term(float &h, float &l, float ph, float pl)
{
    ffd::add22(h, l, ph, pl, h, l);
}

template <class In>
struct Terms;

template <>
struct Terms<InF32> {
    // Four terms of group g (elements 4g..4g+3), masked to [s, e).
    __device__ __forceinline__ static void group(const InF32 &in, int64_t g, int64_t s, int64_t e,
                                                 int64_t total, float2 acc[4])
    {
        const int64_t i0 = 4 * g;
        f32x4 x, y;
        if (i0 + 4 <= total) {
            x = __builtin_nontemporal_load(reinterpret_cast<const f32x4 *>(in.x) + g);
            y = __builtin_nontemporal_load(reinterpret_cast<const f32x4 *>(in.y) + g);
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                x[k] = i0 + k < total ? in.x[i0 + k] : 0.0f;
                y[k] = i0 + k < total ? in.y[i0 + k] : 0.0f;
            }
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            // both factors zeroed outside [s, e): the term is then exactly 0
            // and Add22 leaves the accumulator unchanged
            const bool on = (i0 + k >= s) && (i0 + k < e);
            float p, q;
            ffd::mul12_fma(on ? x[k] : 0.0f, on ? y[k] : 0.0f, p, q);
            accumulate_term(acc[k].x, acc[k].y, p, q);
        }
    }
    __device__ __forceinline__ static void one(const InF32 &in, int64_t i, float2 &acc)
    {
        float p, q;
        ffd::mul12_fma(in.x[i], in.y[i], p, q);
        accumulate_term(acc.x, acc.y, p, q);
    }
};

template <>
struct Terms<InFF> {
    __device__ __forceinline__ static void group(const InFF &in, int64_t g, int64_t s, int64_t e,
                                                 int64_t total, float2 acc[4])
    {
        const int64_t i0 = 4 * g;
        f32x4 xh, xl, yh, yl;
        if (i0 + 4 <= total) {
            xh = __builtin_nontemporal_load(reinterpret_cast<const f32x4 *>(in.xh) + g);
            xl = __builtin_nontemporal_load(reinterpret_cast<const f32x4 *>(in.xl) + g);
            yh = __builtin_nontemporal_load(reinterpret_cast<const f32x4 *>(in.yh) + g);
            yl = __builtin_nontemporal_load(reinterpret_cast<const f32x4 *>(in.yl) + g);
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const bool in_range = i0 + k < total;
                xh[k] = in_range ? in.xh[i0 + k] : 0.0f;
                xl[k] = in_range ? in.xl[i0 + k] : 0.0f;
                yh[k] = in_range ? in.yh[i0 + k] : 0.0f;
                yl[k] = in_range ? in.yl[i0 + k] : 0.0f;
            }
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const bool on = (i0 + k >= s) && (i0 + k < e);
            float ph, pl;
            ffd::mul22<false>(on ? xh[k] : 0.0f, on ? xl[k] : 0.0f, on ? yh[k] : 0.0f,
                              on ? yl[k] : 0.0f, ph, pl);
            accumulate_term(acc[k].x, acc[k].y, ph, pl);
        }
    }
    __device__ __forceinline__ static void one(const InFF &in, int64_t i, float2 &acc)
    {
        float ph, pl;
        ffd::mul22<false>(in.xh[i], in.xl[i], in.yh[i], in.yl[i], ph, pl);
        accumulate_term(acc.x, acc.y, ph, pl);
    }
};

template <>
struct Terms<InSumF32> {
    // term = (x_i, 0): the binary32 value itself
    __device__ __forceinline__ static void group(const InSumF32 &in, int64_t g, int64_t s,
                                                 int64_t e, int64_t total, float2 acc[4])
    {
        const int64_t i0 = 4 * g;
        f32x4 x;
        if (i0 + 4 <= total) {
            x = __builtin_nontemporal_load(reinterpret_cast<const f32x4 *>(in.x) + g);
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k)
                x[k] = i0 + k < total ? in.x[i0 + k] : 0.0f;
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const bool on = (i0 + k >= s) && (i0 + k < e);
            accumulate_term(acc[k].x, acc[k].y, on ? x[k] : 0.0f, 0.0f);
        }
    }
    __device__ __forceinline__ static void one(const InSumF32 &in, int64_t i, float2 &acc)
    {
        accumulate_term(acc.x, acc.y, in.x[i], 0.0f);
    }
};

template <>
struct Terms<InSumFF> {
    __device__ __forceinline__ static void group(const InSumFF &in, int64_t g, int64_t s,
                                                 int64_t e, int64_t total, float2 acc[4])
    {
        const int64_t i0 = 4 * g;
        f32x4 xh, xl;
        if (i0 + 4 <= total) {
            xh = __builtin_nontemporal_load(reinterpret_cast<const f32x4 *>(in.xh) + g);
            xl = __builtin_nontemporal_load(reinterpret_cast<const f32x4 *>(in.xl) + g);
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const bool in_range = i0 + k < total;
                xh[k] = in_range ? in.xh[i0 + k] : 0.0f;
                xl[k] = in_range ? in.xl[i0 + k] : 0.0f;
            }
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const bool on = (i0 + k >= s) && (i0 + k < e);
            accumulate_term(acc[k].x, acc[k].y, on ? xh[k] : 0.0f, on ? xl[k] : 0.0f);
        }
    }
    __device__ __forceinline__ static void one(const InSumFF &in, int64_t i, float2 &acc)
    {
        accumulate_term(acc.x, acc.y, in.xh[i], in.xl[i]);
    }
};

// The persistent launch.  Chunk c goes to workgroup c mod gridDim.x.
// VEC: all planes 16-byte aligned, float4 groups; otherwise element loads.
template <class In, int BLOCK, int UNROLL, bool VEC>
__global__ __launch_bounds__(BLOCK) void dot_batched(In in, const int64_t *__restrict__ offsets,
                                                     int64_t total, int64_t chunk, Workspace w,
                                                     int32_t nvec, float *__restrict__ out_hi,
                                                     float *__restrict__ out_lo)
{
    constexpr int kWaves = BLOCK / 64;
    __shared__ float2 wave_part[kWaves];
    __shared__ int last_flag;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    int64_t nchunks = w.chunk_start[nvec];
    if (nchunks > w.cap)
        nchunks = w.cap;

    for (int64_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const int v = w.chunk_vec[c];
        const int64_t vb = clamp_offset(offsets[v], total);
        const int64_t ve = clamp_offset(offsets[v + 1], total);
        const int64_t c0 = w.chunk_start[v];
        const int64_t c1 = w.chunk_start[v + 1];
        const int64_t s = vb + (c - c0) * chunk;
        const int64_t e = (ve < s + chunk) ? ve : s + chunk;

        float2 acc[4];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            acc[k] = make_float2(0.0f, 0.0f);
        if (VEC) {
            const int64_t g0 = s >> 2;
            const int64_t g1 = (e + 3) >> 2;
            for (int64_t g = g0 + tid; g < g1; g += BLOCK * UNROLL) {
#pragma unroll
                for (int u = 0; u < UNROLL; ++u) {
                    const int64_t gu = g + u * BLOCK;
                    if (gu < g1)
                        Terms<In>::group(in, gu, s, e, total, acc);
                }
            }
        } else {
            for (int64_t i = s + tid; i < e; i += BLOCK)
                Terms<In>::one(in, i, acc[0]);
        }
        float h = acc[0].x, l = acc[0].y;
        ffd::add22(h, l, acc[1].x, acc[1].y, h, l);
        float h2 = acc[2].x, l2 = acc[2].y;
        ffd::add22(h2, l2, acc[3].x, acc[3].y, h2, l2);
        ffd::add22(h, l, h2, l2, h, l);
        ffd::wave_allreduce_add22(h, l);
        if (lane == 0)
            wave_part[wave] = make_float2(h, l);
        __syncthreads();
        if (tid == 0) {
            float th = wave_part[0].x, tl = wave_part[0].y;
#pragma unroll
            for (int k = 1; k < kWaves; ++k)
                ffd::add22(th, tl, wave_part[k].x, wave_part[k].y, th, tl);
            w.partials[c] = make_float2(th, tl);
            __threadfence();   // publish the partial before counting it
            const uint32_t done = atomicAdd(&w.counters[v], 1u);
            last_flag = (static_cast<int64_t>(done) == c1 - c0 - 1);
        }
        __syncthreads();
        if (last_flag && wave == 0) {
            __threadfence();   // observe the other workgroups' partials
            float ph = 0.0f, pl = 0.0f;
            for (int64_t k = c0 + lane; k < c1; k += 64) {
                const float2 p = w.partials[k];
                ffd::add22(ph, pl, p.x, p.y, ph, pl);
            }
            ffd::wave_allreduce_add22(ph, pl);
            if (lane == 0) {
                out_hi[v] = ph;
                out_lo[v] = pl;
            }
        }
        __syncthreads();
    }
}

struct Cfg {
    int block, unroll, grid;
    int64_t chunk;
};

ff_status resolve_cfg(const ff_dot_cfg *cfg, Cfg &out)
{
    out.block = 256;
    out.chunk = 16384;
    out.grid = 0;
    out.unroll = 2;
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
    if (out.unroll != 1 && out.unroll != 2 && out.unroll != 4)
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
    if (hipGetDevice(&dev) == hipSuccess)
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    return 8 * (cus > 0 ? cus : 256);
}

template <class In, int BLOCK, int UNROLL>
void launch_main(bool vec, int grid, hipStream_t st, const In &in, const int64_t *offsets,
                 int64_t total, int64_t chunk, const Workspace &w, int32_t nvec, float *oh,
                 float *ol)
{
    if (vec)
        hipLaunchKernelGGL((dot_batched<In, BLOCK, UNROLL, true>), dim3(grid), dim3(BLOCK), 0, st,
                           in, offsets, total, chunk, w, nvec, oh, ol);
    else
        hipLaunchKernelGGL((dot_batched<In, BLOCK, 1, false>), dim3(grid), dim3(BLOCK), 0, st, in,
                           offsets, total, chunk, w, nvec, oh, ol);
}

template <class In>
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
    hipLaunchKernelGGL(dot_plan, dim3(1), dim3(kPlanBlock), 0, st, offsets, nvec, total, cfg.chunk,
                       w, out_hi, out_lo);
    if (cfg.block == 256) {
        if (cfg.unroll == 1)
            launch_main<In, 256, 1>(vec, grid, st, in, offsets, total, cfg.chunk, w, nvec, out_hi, out_lo);
        else if (cfg.unroll == 2)
            launch_main<In, 256, 2>(vec, grid, st, in, offsets, total, cfg.chunk, w, nvec, out_hi, out_lo);
        else
            launch_main<In, 256, 4>(vec, grid, st, in, offsets, total, cfg.chunk, w, nvec, out_hi, out_lo);
    } else {
        if (cfg.unroll == 1)
            launch_main<In, 512, 1>(vec, grid, st, in, offsets, total, cfg.chunk, w, nvec, out_hi, out_lo);
        else if (cfg.unroll == 2)
            launch_main<In, 512, 2>(vec, grid, st, in, offsets, total, cfg.chunk, w, nvec, out_hi, out_lo);
        else
            launch_main<In, 512, 4>(vec, grid, st, in, offsets, total, cfg.chunk, w, nvec, out_hi, out_lo);
    }
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
    static const int kUnrolls[] = {1, 2, 4};
    static const int kChunks[] = {4096, 8192, 16384, 32768, 65536};
    static const int kPerCu[] = {2, 4, 8, 16};
    hipStream_t st = ffh::as_stream(stream);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess)
        return ffh::hip_failure(hipGetLastError());
    if (hipEventCreate(&e1) != hipSuccess) {
        hipEventDestroy(e0);
        return ffh::hip_failure(hipGetLastError());
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
                    hipEventRecord(e0, st);
                    for (int r = 0; r < reps && status == FF_OK; ++r)
                        status = ff_dot_batched(x, y, offsets, nvec, total_len, &c, ws, ws_bytes,
                                                out_hi, out_lo, stream);
                    hipEventRecord(e1, st);
                    if (status != FF_OK)
                        goto done;
                    if (hipEventSynchronize(e1) != hipSuccess) {
                        status = ffh::hip_failure(hipGetLastError());
                        goto done;
                    }
                    float ms = 0.0f;
                    hipEventElapsedTime(&ms, e0, e1);
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
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    return status;
}

} // extern "C"
