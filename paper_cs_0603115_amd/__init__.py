"""Float-float (hi + lo binary32) arithmetic on AMD Instinct MI355X.

A thin Python binding over the C ABI of ``libff.so`` (``include/ff.h``):
every function here only checks and marshals arguments; every arithmetic
step runs in the library's HIP kernels.  PyTorch provides device memory and
streams.

A float-float tensor is a float32 tensor of shape ``(2, *shape)`` whose
plane 0 holds the high words and plane 1 the low words, each plane
contiguous (structure of arrays).  Work is enqueued on the current torch
stream unless ``stream`` is given.
"""
from __future__ import annotations

import ctypes
import functools
import inspect

import torch

from ._lib import (GEMM_FMA_LOOP, GEMM_SLICED_BF16, GEMM_SLICED_I8, MATVEC_FAST, MATVEC_PLAIN,
                   DotCfg, FFError, check, lib)

__all__ = [
    "lib", "FFError", "DotCfg", "build_info",
    "ff_add", "ff_sub", "ff_mul", "ff_mul_dekker", "ff_div", "ff_copy",
    "ff_add_accurate", "ff_sub_accurate", "ff_mul_accurate", "ff_div_accurate",
    "ff_add12", "ff_mul12", "f32_add", "f32_mul", "f32_mad",
    "ff_horner_f32", "ff_horner_comp", "ff_horner_ff",
    "ff_dot_batched", "ff_dot_batched_noalloc", "ff_dot_ff_batched",
    "ff_dot_batched_workspace_size",
    "ff_sum_batched", "ff_sum_ff_batched", "ff_dot2_batched", "ff_sum2_batched",
    "ff_matvec", "ff_matvec_backward", "ff_matvec_backward_workspace_size", "ff_dot_backward",
    "ff_dot_batched_backward", "ff_dot_batched_backward_workspace_size",
    "MATVEC_FAST", "MATVEC_PLAIN",
    "ff_gemm", "ff_gemm_workspace_size", "GEMM_FMA_LOOP", "GEMM_SLICED_BF16", "GEMM_SLICED_I8",
    "ff_empty", "ff_zeros", "ff_from_f64", "ff_to_f64",
    "add", "sub", "mul", "div", "dot_batched", "gemm", "matvec", "from_float64", "to_float64",
]


def build_info() -> str:
    """How the loaded library was built (target, numerics flags)."""
    return lib.ff_build_info().decode()


def _torch_stream(stream):
    if isinstance(stream, torch.cuda.Stream):
        return stream
    return torch.cuda.ExternalStream(int(stream))


def _on_stream(fn):
    """Run a wrapper with ``stream`` (when given) as torch's current stream,
    so that the outputs and workspaces it allocates belong to the stream its
    kernels are enqueued on: the caching allocator then cannot hand that
    memory to other work before those kernels are done with it."""
    sig = inspect.signature(fn)

    @functools.wraps(fn)
    def run(*args, **kwargs):
        stream = sig.bind_partial(*args, **kwargs).arguments.get("stream")
        if stream is None:
            return fn(*args, **kwargs)
        with torch.cuda.stream(_torch_stream(stream)):
            return fn(*args, **kwargs)

    return run


def _stream_handle(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _check_ff(t: torch.Tensor, name: str) -> None:
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float32:
        raise TypeError(f"{name}: expected a float32 tensor")
    if t.dim() < 1 or t.shape[0] != 2:
        raise ValueError(f"{name}: a float-float tensor has shape (2, ...), got {tuple(t.shape)}")
    if not t.is_cuda:
        raise ValueError(f"{name}: must be on a HIP device (libff runs on the GPU only)")
    if not (t[0].is_contiguous() and t[1].is_contiguous()):
        raise ValueError(f"{name}: each plane must be contiguous")


def _planes(t: torch.Tensor):
    return ctypes.c_void_p(t[0].data_ptr()), ctypes.c_void_p(t[1].data_ptr())


# Plane stride granule of ff_empty / ff_zeros, in binary32 words (4 KiB).
PLANE_ALIGN = 1024


def _planar(alloc, shape, device) -> torch.Tensor:
    """A (2, *shape) float32 tensor whose two planes are each contiguous and
    start a multiple of 4 KiB apart.  The allocator aligns the first plane,
    so both are: a wavefront's access of 64 consecutive words of either plane
    is then one aligned 256-byte segment.  (In a plain (2, n) tensor the low
    plane starts 4n bytes after the high one; unless n is a multiple of 64
    every such access straddles two segments, which cost the streaming
    kernels up to 8 % of their rate on MI355X.)"""
    shape = tuple(int(d) for d in shape)
    numel = 1
    for d in shape:
        numel *= d
    stride = -(-max(numel, 1) // PLANE_ALIGN) * PLANE_ALIGN
    base = alloc(2 * stride, dtype=torch.float32, device=device)
    inner = []
    acc = 1
    for d in reversed(shape):
        inner.append(acc)
        acc *= max(d, 1)
    return base.as_strided((2, *shape), (stride, *reversed(inner)))


def ff_empty(shape, device="cuda") -> torch.Tensor:
    """Uninitialised float-float tensor of the given value shape (planes
    aligned as described in _planar)."""
    return _planar(torch.empty, shape, device)


def ff_zeros(shape, device="cuda") -> torch.Tensor:
    """Float-float zeros of the given value shape (planes aligned as
    described in _planar)."""
    return _planar(torch.zeros, shape, device)


def _elementwise(name: str, a: torch.Tensor, b: torch.Tensor, out, stream) -> torch.Tensor:
    _check_ff(a, "a")
    _check_ff(b, "b")
    if a.shape != b.shape:
        raise ValueError(f"{name}: operand shapes differ: {tuple(a.shape)} vs {tuple(b.shape)}")
    if a.device != b.device:
        raise ValueError(f"{name}: operands on different devices")
    if out is None:
        out = ff_empty(a.shape[1:], device=a.device)
    else:
        _check_ff(out, "out")
        if out.shape != a.shape:
            raise ValueError(f"{name}: out has shape {tuple(out.shape)}")
    n = a[0].numel()
    ah, al = _planes(a)
    bh, bl = _planes(b)
    rh, rl = _planes(out)
    with torch.cuda.device(a.device):
        check(name, getattr(lib, name)(ah, al, bh, bl, rh, rl, n, _stream_handle(stream)))
    return out


@_on_stream
def ff_add(a, b, out=None, stream=None):
    """Float-float sum a + b (Add22, section 4.1)."""
    return _elementwise("ff_add", a, b, out, stream)


@_on_stream
def ff_sub(a, b, out=None, stream=None):
    """Float-float difference a - b (Add22 of a and -b)."""
    return _elementwise("ff_sub", a, b, out, stream)


@_on_stream
def ff_mul(a, b, out=None, stream=None):
    """Float-float product a * b (Mul22, FMA TwoProd)."""
    return _elementwise("ff_mul", a, b, out, stream)


@_on_stream
def ff_mul_dekker(a, b, out=None, stream=None):
    """Float-float product a * b (Mul22 with Dekker's Split-based Mul12)."""
    return _elementwise("ff_mul_dekker", a, b, out, stream)


@_on_stream
def ff_div(a, b, out=None, stream=None):
    """Float-float quotient a / b (Div22, Dekker's div2)."""
    return _elementwise("ff_div", a, b, out, stream)


@_on_stream
def ff_add_accurate(a, b, out=None, stream=None):
    """Cancellation-safe float-float sum (AccurateDWPlusDW of Joldes, Muller
    and Popescu): relative error below 3u^2/(1 - 4u), u = 2^-24, also when
    a and b cancel."""
    return _elementwise("ff_add_accurate", a, b, out, stream)


@_on_stream
def ff_sub_accurate(a, b, out=None, stream=None):
    """Cancellation-safe float-float difference a - b."""
    return _elementwise("ff_sub_accurate", a, b, out, stream)


@_on_stream
def ff_mul_accurate(a, b, out=None, stream=None):
    """FMA-based float-float product (DWTimesDW3 of Joldes, Muller and
    Popescu): relative error at most 5u^2, u = 2^-24."""
    return _elementwise("ff_mul_accurate", a, b, out, stream)


@_on_stream
def ff_div_accurate(a, b, out=None, stream=None):
    """Reciprocal-based float-float quotient a / b (DWDivDW3 of Joldes,
    Muller and Popescu): relative error at most 9.8u^2, one division per
    element; for 2^-126 < |b_hi| < 2^126."""
    return _elementwise("ff_div_accurate", a, b, out, stream)


@_on_stream
def ff_copy(src: torch.Tensor, dst: torch.Tensor, stream=None) -> torch.Tensor:
    """dst <- src for float32 tensors (the bandwidth probe kernel)."""
    if src.dtype != torch.float32 or dst.dtype != torch.float32:
        raise TypeError("ff_copy: float32 tensors expected")
    if not (src.is_contiguous() and dst.is_contiguous()) or src.numel() != dst.numel():
        raise ValueError("ff_copy: contiguous tensors of equal size expected")
    if not src.is_cuda:
        raise ValueError("ff_copy: tensors must be on a HIP device")
    with torch.cuda.device(src.device):
        check("ff_copy", lib.ff_copy(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                                     src.numel(), _stream_handle(stream)))
    return dst


# ------------------------------------------- error-free transforms, binary32

def _f32_operands(name: str, *ts: torch.Tensor):
    for k, t in enumerate(ts):
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float32:
            raise TypeError(f"{name}: operand {k} must be a float32 tensor")
        if not t.is_cuda:
            raise ValueError(f"{name}: operands must be on a HIP device")
        if not t.is_contiguous():
            raise ValueError(f"{name}: operands must be contiguous")
        if t.shape != ts[0].shape or t.device != ts[0].device:
            raise ValueError(f"{name}: operands differ in shape or device")


def _check_pair_out(name: str, out: torch.Tensor, a: torch.Tensor) -> None:
    _check_ff(out, "out")
    if out.shape != (2, *a.shape) or out.device != a.device:
        raise ValueError(f"{name}: out must have shape {(2, *a.shape)} on {a.device}")


def _ptr(t: torch.Tensor) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


@_on_stream
def ff_add12(a: torch.Tensor, b: torch.Tensor, out=None, stream=None) -> torch.Tensor:
    """Add12 theorem (section 4.1) elementwise on binary32 tensors: the
    float-float result (s, r) with s = a (+) b and s + r = a + b exactly."""
    _f32_operands("ff_add12", a, b)
    out = ff_empty(a.shape, device=a.device) if out is None else out
    _check_pair_out("ff_add12", out, a)
    with torch.cuda.device(a.device):
        check("ff_add12", lib.ff_add12(_ptr(a), _ptr(b), *_planes(out), a.numel(),
                                       _stream_handle(stream)))
    return out


@_on_stream
def ff_mul12(a: torch.Tensor, b: torch.Tensor, dekker: bool = False, out=None,
             stream=None) -> torch.Tensor:
    """Exact products elementwise: (x, y) with x = a (x) b, x + y = a b, by
    FMA TwoProd or (dekker=True) by the Mul12 theorem's Split algorithm."""
    name = "ff_mul12_dekker" if dekker else "ff_mul12"
    _f32_operands(name, a, b)
    out = ff_empty(a.shape, device=a.device) if out is None else out
    _check_pair_out(name, out, a)
    with torch.cuda.device(a.device):
        check(name, getattr(lib, name)(_ptr(a), _ptr(b), *_planes(out), a.numel(),
                                       _stream_handle(stream)))
    return out


def _f32_binary(name: str, a, b, out, stream) -> torch.Tensor:
    _f32_operands(name, a, b)
    out = torch.empty_like(a) if out is None else out
    _f32_operands(name, a, out)
    with torch.cuda.device(a.device):
        check(name, getattr(lib, name)(_ptr(a), _ptr(b), _ptr(out), a.numel(),
                                       _stream_handle(stream)))
    return out


@_on_stream
def f32_add(a, b, out=None, stream=None) -> torch.Tensor:
    """Binary32 a (+) b: the reference operator of the paper's tables."""
    return _f32_binary("ff_f32_add", a, b, out, stream)


@_on_stream
def f32_mul(a, b, out=None, stream=None) -> torch.Tensor:
    """Binary32 a (x) b: the reference operator of the paper's tables."""
    return _f32_binary("ff_f32_mul", a, b, out, stream)


@_on_stream
def f32_mad(a, b, c, out=None, stream=None) -> torch.Tensor:
    """Binary32 fma(a, b, c), one rounding: the tables' multiply-add."""
    _f32_operands("ff_f32_mad", a, b, c)
    out = torch.empty_like(a) if out is None else out
    _f32_operands("ff_f32_mad", a, out)
    with torch.cuda.device(a.device):
        check("ff_f32_mad", lib.ff_f32_mad(_ptr(a), _ptr(b), _ptr(c), _ptr(out), a.numel(),
                                           _stream_handle(stream)))
    return out


# ----------------------------------------------------------------- conversions

@_on_stream
def ff_from_f64(x: torch.Tensor, out=None, stream=None) -> torch.Tensor:
    """binary64 tensor -> float-float tensor (2, *x.shape): hi = fl32(x),
    lo = fl32(x - hi), on the device."""
    if not isinstance(x, torch.Tensor) or x.dtype != torch.float64 or not x.is_cuda:
        raise TypeError("ff_from_f64: expected a float64 tensor on a HIP device")
    if not x.is_contiguous():
        raise ValueError("ff_from_f64: x must be contiguous")
    out = ff_empty(x.shape, device=x.device) if out is None else out
    _check_ff(out, "out")
    if tuple(out.shape) != (2, *x.shape) or out.device != x.device:
        raise ValueError(f"ff_from_f64: out must have shape {(2, *x.shape)} on {x.device}")
    with torch.cuda.device(x.device):
        check("ff_from_f64", lib.ff_from_f64(_ptr(x), *_planes(out), x.numel(),
                                             _stream_handle(stream)))
    return out


@_on_stream
def ff_to_f64(a: torch.Tensor, out=None, stream=None) -> torch.Tensor:
    """float-float tensor -> binary64 tensor: (double) hi + (double) lo, one
    rounding, on the device."""
    _check_ff(a, "a")
    shape = tuple(a.shape[1:])
    out = torch.empty(shape, dtype=torch.float64, device=a.device) if out is None else out
    if not isinstance(out, torch.Tensor) or out.dtype != torch.float64 or \
            tuple(out.shape) != shape or out.device != a.device or not out.is_contiguous():
        raise ValueError(f"ff_to_f64: out must be a contiguous float64 tensor of shape {shape}")
    with torch.cuda.device(a.device):
        check("ff_to_f64", lib.ff_to_f64(*_planes(a), _ptr(out), out.numel(),
                                         _stream_handle(stream)))
    return out


# ------------------------------------------------------- polynomial evaluation

def _coefficients(name: str, coef: torch.Tensor, ff: bool):
    """Device pointers (hi, lo or None) and degree of a coefficient tensor:
    binary32 (degree + 1,) or, when ff is allowed, float-float (2, degree + 1)."""
    if not isinstance(coef, torch.Tensor) or coef.dtype != torch.float32 or not coef.is_cuda:
        raise TypeError(f"{name}: coefficients must be a float32 tensor on a HIP device")
    if coef.dim() == 1:
        if not coef.is_contiguous():
            raise ValueError(f"{name}: coefficients must be contiguous")
        hi, lo, count = coef, None, coef.numel()
    elif ff and coef.dim() == 2 and coef.shape[0] == 2:
        _check_ff(coef, "coef")
        hi, lo, count = coef[0], coef[1], coef.shape[1]
    else:
        raise ValueError(f"{name}: coefficients of shape {tuple(coef.shape)}")
    if count < 1:
        raise ValueError(f"{name}: a polynomial needs at least one coefficient")
    return _ptr(hi), (None if lo is None else _ptr(lo)), count - 1


def _horner_f32(name, coef, x, out, stream):
    ch, _, degree = _coefficients(name, coef, ff=False)
    _f32_operands(name, x)
    if coef.device != x.device:
        raise ValueError(f"{name}: coefficients and points on different devices")
    out = torch.empty_like(x) if out is None else out
    _f32_operands(name, x, out)
    with torch.cuda.device(x.device):
        check(name, getattr(lib, name)(ch, degree, _ptr(x), _ptr(out), x.numel(),
                                       _stream_handle(stream)))
    return out


@_on_stream
def ff_horner_f32(coef, x, out=None, stream=None) -> torch.Tensor:
    """Horner's rule in binary32: sum_i coef[i] x^i at every point of x."""
    return _horner_f32("ff_horner_f32", coef, x, out, stream)


@_on_stream
def ff_horner_comp(coef, x, out=None, stream=None) -> torch.Tensor:
    """Compensated Horner (Graillat, Langlois and Louvet) at every point of
    x: binary32 results as accurate as Horner's rule in twice the working
    precision, rounded once."""
    return _horner_f32("ff_horner_comp", coef, x, out, stream)


@_on_stream
def ff_horner_ff(coef, x, out=None, stream=None, ff_points: bool = True) -> torch.Tensor:
    """Float-float Horner (Mul22 then Add22 per step).  coef: binary32
    (degree + 1,) or float-float (2, degree + 1); x: a float-float tensor
    (2, ...) of points, or with ff_points=False binary32 points of any shape.
    Returns a float-float tensor (2, *points shape)."""
    name = "ff_horner_ff"
    ch, cl, degree = _coefficients(name, coef, ff=True)
    if ff_points:
        _check_ff(x, "x")
        xh, xl = _planes(x)
        shape = tuple(x.shape[1:])
    else:
        _f32_operands(name, x)
        xh, xl, shape = _ptr(x), None, tuple(x.shape)
    dev = coef.device
    if x.device != dev:
        raise ValueError(f"{name}: coefficients and points on different devices")
    out = ff_empty(shape, device=dev) if out is None else out
    _check_ff(out, "out")
    if tuple(out.shape) != (2, *shape) or out.device != dev:
        raise ValueError(f"{name}: out must have shape {(2, *shape)} on {dev}")
    n = 1
    for d in shape:
        n *= d
    with torch.cuda.device(dev):
        check(name, lib.ff_horner_ff(ch, cl, degree, xh, xl, *_planes(out), n,
                                     _stream_handle(stream)))
    return out


# ------------------------------------------------------------------ reductions

def _cfg_ptr(cfg):
    if cfg is None:
        return None
    if isinstance(cfg, DotCfg):
        return ctypes.byref(cfg)
    return ctypes.byref(DotCfg(*cfg))


def ff_dot_batched_workspace_size(total_len: int, nvec: int, cfg=None) -> int:
    """Workspace bytes for a batched dot over ``nvec`` vectors of ``total_len``
    elements in all."""
    return int(lib.ff_dot_batched_workspace_size(int(total_len), int(nvec), _cfg_ptr(cfg)))


def _check_offsets(offsets: torch.Tensor, device) -> int:
    if offsets.dtype != torch.int64 or offsets.dim() != 1 or not offsets.is_contiguous():
        raise ValueError("offsets: contiguous int64 vector of nvec + 1 entries expected")
    if offsets.device != device:
        raise ValueError("offsets must be on the same device as the data")
    return offsets.numel() - 1


def _workspace(nbytes: int, device, workspace):
    if workspace is None:
        return torch.empty(max(nbytes, 1), dtype=torch.uint8, device=device)
    if workspace.device != device or workspace.numel() * workspace.element_size() < nbytes:
        raise ValueError("workspace too small or on another device")
    return workspace


@_on_stream
def ff_dot_batched(x: torch.Tensor, y: torch.Tensor, offsets: torch.Tensor, cfg=None,
                   out=None, workspace=None, stream=None) -> torch.Tensor:
    """Float-float dots of binary32 vectors: out[:, v] = sum of x*y over
    [offsets[v], offsets[v+1]) (TwoProd terms, Add22 accumulation).
    Returns a float-float tensor of shape (2, nvec)."""
    for t, name in ((x, "x"), (y, "y")):
        if t.dtype != torch.float32 or t.dim() != 1 or not t.is_contiguous() or not t.is_cuda:
            raise ValueError(f"{name}: contiguous float32 vector on a HIP device expected")
    if x.numel() != y.numel():
        raise ValueError("x and y differ in length")
    nvec = _check_offsets(offsets, x.device)
    out = ff_empty((nvec,), device=x.device) if out is None else out
    _check_ff(out, "out")
    nbytes = ff_dot_batched_workspace_size(x.numel(), nvec, cfg)
    ws = _workspace(nbytes, x.device, workspace)
    oh, ol = _planes(out)
    with torch.cuda.device(x.device):
        check("ff_dot_batched", lib.ff_dot_batched(
            ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
            ctypes.c_void_p(offsets.data_ptr()), nvec, x.numel(), _cfg_ptr(cfg),
            ctypes.c_void_p(ws.data_ptr()), ws.numel(), oh, ol, _stream_handle(stream)))
    return out


@_on_stream
def ff_dot_batched_noalloc(x: torch.Tensor, y: torch.Tensor, offsets: torch.Tensor, cfg=None,
                           out=None, stream=None) -> torch.Tensor:
    """ff_dot_batched through the entry point that takes no workspace (its
    scratch is a static device array of the library, shared by every call on
    the device: calls that may overlap there race).  Allocates the output
    only when ``out`` is None."""
    for t, name in ((x, "x"), (y, "y")):
        if t.dtype != torch.float32 or t.dim() != 1 or not t.is_contiguous() or not t.is_cuda:
            raise ValueError(f"{name}: contiguous float32 vector on a HIP device expected")
    if x.numel() != y.numel():
        raise ValueError("x and y differ in length")
    nvec = _check_offsets(offsets, x.device)
    out = ff_empty((nvec,), device=x.device) if out is None else out
    _check_ff(out, "out")
    oh, ol = _planes(out)
    with torch.cuda.device(x.device):
        check("ff_dot_batched_noalloc", lib.ff_dot_batched_noalloc(
            ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
            ctypes.c_void_p(offsets.data_ptr()), nvec, x.numel(), _cfg_ptr(cfg), oh, ol,
            _stream_handle(stream)))
    return out


@_on_stream
def ff_dot2_batched(x: torch.Tensor, y: torch.Tensor, offsets: torch.Tensor, cfg=None,
                    out=None, workspace=None, stream=None) -> torch.Tensor:
    """Compensated dots (Dot2 of Ogita, Rump and Oishi) of binary32 vectors:
    out[0, v] is the binary32 Dot2 result of [offsets[v], offsets[v+1]),
    out[1, v] the remainder of its final rounding.  Returns (2, nvec)."""
    for t, name in ((x, "x"), (y, "y")):
        if t.dtype != torch.float32 or t.dim() != 1 or not t.is_contiguous() or not t.is_cuda:
            raise ValueError(f"{name}: contiguous float32 vector on a HIP device expected")
    if x.numel() != y.numel():
        raise ValueError("x and y differ in length")
    nvec = _check_offsets(offsets, x.device)
    out = ff_empty((nvec,), device=x.device) if out is None else out
    _check_ff(out, "out")
    ws = _workspace(ff_dot_batched_workspace_size(x.numel(), nvec, cfg), x.device, workspace)
    oh, ol = _planes(out)
    with torch.cuda.device(x.device):
        check("ff_dot2_batched", lib.ff_dot2_batched(
            ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
            ctypes.c_void_p(offsets.data_ptr()), nvec, x.numel(), _cfg_ptr(cfg),
            ctypes.c_void_p(ws.data_ptr()), ws.numel(), oh, ol, _stream_handle(stream)))
    return out


@_on_stream
def ff_sum2_batched(x: torch.Tensor, offsets: torch.Tensor, cfg=None, out=None, workspace=None,
                    stream=None) -> torch.Tensor:
    """Compensated sums (Sum2 of Ogita, Rump and Oishi) of binary32
    segments; same result layout as ff_dot2_batched."""
    if x.dtype != torch.float32 or x.dim() != 1 or not x.is_contiguous() or not x.is_cuda:
        raise ValueError("x: contiguous float32 vector on a HIP device expected")
    nvec = _check_offsets(offsets, x.device)
    out = ff_empty((nvec,), device=x.device) if out is None else out
    _check_ff(out, "out")
    ws = _workspace(ff_dot_batched_workspace_size(x.numel(), nvec, cfg), x.device, workspace)
    oh, ol = _planes(out)
    with torch.cuda.device(x.device):
        check("ff_sum2_batched", lib.ff_sum2_batched(
            ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(offsets.data_ptr()), nvec, x.numel(),
            _cfg_ptr(cfg), ctypes.c_void_p(ws.data_ptr()), ws.numel(), oh, ol,
            _stream_handle(stream)))
    return out


@_on_stream
def ff_dot_ff_batched(x: torch.Tensor, y: torch.Tensor, offsets: torch.Tensor, cfg=None,
                      out=None, workspace=None, stream=None) -> torch.Tensor:
    """Float-float dots of float-float vectors (Mul22 terms, Add22
    accumulation); x and y have shape (2, total).  Returns (2, nvec)."""
    _check_ff(x, "x")
    _check_ff(y, "y")
    if x.shape != y.shape or x.dim() != 2:
        raise ValueError("x and y must both have shape (2, total)")
    nvec = _check_offsets(offsets, x.device)
    out = ff_empty((nvec,), device=x.device) if out is None else out
    _check_ff(out, "out")
    total = x.shape[1]
    nbytes = ff_dot_batched_workspace_size(total, nvec, cfg)
    ws = _workspace(nbytes, x.device, workspace)
    xh, xl = _planes(x)
    yh, yl = _planes(y)
    oh, ol = _planes(out)
    with torch.cuda.device(x.device):
        check("ff_dot_ff_batched", lib.ff_dot_ff_batched(
            xh, xl, yh, yl, ctypes.c_void_p(offsets.data_ptr()), nvec, total, _cfg_ptr(cfg),
            ctypes.c_void_p(ws.data_ptr()), ws.numel(), oh, ol, _stream_handle(stream)))
    return out


@_on_stream
def ff_sum_batched(x: torch.Tensor, offsets: torch.Tensor, cfg=None, out=None, workspace=None,
                   stream=None) -> torch.Tensor:
    """Float-float sums of binary32 segments [offsets[v], offsets[v+1]) of x
    (Add22 accumulation).  Returns (2, nvec)."""
    if x.dtype != torch.float32 or x.dim() != 1 or not x.is_contiguous() or not x.is_cuda:
        raise ValueError("x: contiguous float32 vector on a HIP device expected")
    nvec = _check_offsets(offsets, x.device)
    out = ff_empty((nvec,), device=x.device) if out is None else out
    _check_ff(out, "out")
    ws = _workspace(ff_dot_batched_workspace_size(x.numel(), nvec, cfg), x.device, workspace)
    oh, ol = _planes(out)
    with torch.cuda.device(x.device):
        check("ff_sum_batched", lib.ff_sum_batched(
            ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(offsets.data_ptr()), nvec, x.numel(),
            _cfg_ptr(cfg), ctypes.c_void_p(ws.data_ptr()), ws.numel(), oh, ol,
            _stream_handle(stream)))
    return out


@_on_stream
def ff_sum_ff_batched(x: torch.Tensor, offsets: torch.Tensor, cfg=None, out=None,
                      workspace=None, stream=None) -> torch.Tensor:
    """Float-float sums of float-float segments of x (shape (2, total))."""
    _check_ff(x, "x")
    if x.dim() != 2:
        raise ValueError("x must have shape (2, total)")
    nvec = _check_offsets(offsets, x.device)
    out = ff_empty((nvec,), device=x.device) if out is None else out
    _check_ff(out, "out")
    total = x.shape[1]
    ws = _workspace(ff_dot_batched_workspace_size(total, nvec, cfg), x.device, workspace)
    xh, xl = _planes(x)
    oh, ol = _planes(out)
    with torch.cuda.device(x.device):
        check("ff_sum_ff_batched", lib.ff_sum_ff_batched(
            xh, xl, ctypes.c_void_p(offsets.data_ptr()), nvec, total, _cfg_ptr(cfg),
            ctypes.c_void_p(ws.data_ptr()), ws.numel(), oh, ol, _stream_handle(stream)))
    return out


# ------------------------------------------------------------ differentiation

def _null():
    return ctypes.c_void_p(0)


def _check_matrix(A: torch.Tensor):
    """A float-float matrix (2, M, N): each plane row-major with unit column
    stride and a common leading dimension (row stride) >= N."""
    if not isinstance(A, torch.Tensor) or A.dtype != torch.float32:
        raise TypeError("A: expected a float32 tensor")
    if A.dim() != 3 or A.shape[0] != 2:
        raise ValueError(f"A must have shape (2, M, N), got {tuple(A.shape)}")
    if not A.is_cuda:
        raise ValueError("A: must be on a HIP device (libff runs on the GPU only)")
    M, N = A.shape[1], A.shape[2]
    if (N > 1 and A.stride(2) != 1) or (M > 1 and A.stride(1) < N):
        raise ValueError("A: each plane must be row-major with unit column stride")
    lda = A.stride(1) if M > 1 else max(N, 1)
    return M, N, lda


@_on_stream
def ff_matvec(A: torch.Tensor, x: torch.Tensor, algo: int = MATVEC_FAST, out=None,
              stream=None) -> torch.Tensor:
    """y = A x for a float-float matrix A (2, M, N) and vector x (2, N)."""
    M, N, lda = _check_matrix(A)
    _check_ff(x, "x")
    if x.shape != (2, N):
        raise ValueError(f"x must have shape (2, {N})")
    out = ff_empty((M,), device=A.device) if out is None else out
    _check_ff(out, "out")
    Ah, Al = _planes(A)
    xh, xl = _planes(x)
    yh, yl = _planes(out)
    with torch.cuda.device(A.device):
        check("ff_matvec", lib.ff_matvec(M, N, Ah, Al, lda, xh, xl, yh, yl, int(algo),
                                         _stream_handle(stream)))
    return out


def ff_matvec_backward_workspace_size(M: int, N: int, algo: int = MATVEC_FAST) -> int:
    """Workspace bytes ff_matvec_backward needs for an M x N matrix."""
    return int(lib.ff_matvec_backward_workspace_size(M, N, int(algo)))


@_on_stream
def ff_matvec_backward(A: torch.Tensor, x: torch.Tensor, g: torch.Tensor, want_dA: bool = True,
                       want_dx: bool = True, algo: int = MATVEC_FAST, dA_out=None, dx_out=None,
                       workspace=None, stream=None):
    """Backward pass of y = A x for the upstream float-float gradient g (2, M):
    returns (dA, dx) = (g x^T, A^T g); a gradient not wanted is None.
    dA_out (2, M, N) and dx_out (2, N) receive the gradients when given;
    workspace (uint8, at least ff_matvec_backward_workspace_size bytes)
    replaces the per-call allocation."""
    M, N, lda = _check_matrix(A)
    _check_ff(x, "x")
    _check_ff(g, "g")
    if x.shape != (2, N) or g.shape != (2, M):
        raise ValueError("shape mismatch between A, x and g")
    dA = (ff_empty((M, N), device=A.device) if dA_out is None else dA_out) if want_dA else None
    dx = (ff_empty((N,), device=A.device) if dx_out is None else dx_out) if want_dx else None
    if dA is not None:
        _check_ff(dA, "dA_out")
        if dA.shape != (2, M, N):
            raise ValueError(f"dA_out must have shape (2, {M}, {N})")
    if dx is not None:
        _check_ff(dx, "dx_out")
        if dx.shape != (2, N):
            raise ValueError(f"dx_out must have shape (2, {N})")
    nbytes = ff_matvec_backward_workspace_size(M, N, algo) if want_dx else 0
    ws = _workspace(max(nbytes, 16), A.device, workspace)
    Ah, Al = _planes(A)
    xh, xl = _planes(x)
    gh, gl = _planes(g)
    dAh, dAl = _planes(dA) if want_dA else (_null(), _null())
    dxh, dxl = _planes(dx) if want_dx else (_null(), _null())
    with torch.cuda.device(A.device):
        check("ff_matvec_backward", lib.ff_matvec_backward(
            M, N, Ah, Al, lda, xh, xl, gh, gl, dAh, dAl, N, dxh, dxl, int(algo),
            ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_handle(stream)))
    return dA, dx


@_on_stream
def ff_dot_backward(g: torch.Tensor, x: torch.Tensor, y: torch.Tensor, want_dx: bool = True,
                    want_dy: bool = True, dx_out=None, dy_out=None, stream=None):
    """Backward pass of s = sum x_i y_i for an upstream float-float gradient
    g (shape (2,) or (2, 1)): returns (g y, g x) (elementwise Mul22), written
    into dx_out / dy_out (shaped like x) when given."""
    _check_ff(g, "g")
    _check_ff(x, "x")
    _check_ff(y, "y")
    if g[0].numel() != 1 or x.shape != y.shape:
        raise ValueError("g must hold one float-float value and x, y agree in shape")
    n = x[0].numel()
    dx = (ff_empty(x.shape[1:], device=x.device) if dx_out is None else dx_out) if want_dx else None
    dy = (ff_empty(y.shape[1:], device=y.device) if dy_out is None else dy_out) if want_dy else None
    for t, name in ((dx, "dx_out"), (dy, "dy_out")):
        if t is not None:
            _check_ff(t, name)
            if t.shape != x.shape or t.device != x.device:
                raise ValueError(f"{name} must have shape {tuple(x.shape)} on {x.device}")
    g = g.reshape(2, 1).contiguous()
    gh, gl = _planes(g)
    xh, xl = _planes(x)
    yh, yl = _planes(y)
    dxh, dxl = _planes(dx) if want_dx else (_null(), _null())
    dyh, dyl = _planes(dy) if want_dy else (_null(), _null())
    with torch.cuda.device(x.device):
        check("ff_dot_backward", lib.ff_dot_backward(gh, gl, xh, xl, yh, yl, dxh, dxl, dyh, dyl, n,
                                                     _stream_handle(stream)))
    return dx, dy


def _ff_or_f32_planes(t: torch.Tensor, name: str):
    """(hi, lo or NULL, n) of a float-float (2, n) or binary32 (n,) vector."""
    if isinstance(t, torch.Tensor) and t.dtype == torch.float32 and t.dim() == 1:
        if not t.is_cuda or not t.is_contiguous():
            raise ValueError(f"{name}: contiguous float32 vector on a HIP device expected")
        return _ptr(t), _null(), t.numel()
    _check_ff(t, name)
    if t.dim() != 2:
        raise ValueError(f"{name}: float-float vector (2, n) or binary32 vector (n,) expected")
    hi, lo = _planes(t)
    return hi, lo, t.shape[1]


def ff_dot_batched_backward_workspace_size(total: int) -> int:
    """Workspace bytes ff_dot_batched_backward needs for `total` elements."""
    return int(lib.ff_dot_batched_backward_workspace_size(int(total)))


@_on_stream
def ff_dot_batched_backward(g: torch.Tensor, x: torch.Tensor, y: torch.Tensor,
                            offsets: torch.Tensor, want_dx: bool = True, want_dy: bool = True,
                            dx_out=None, dy_out=None, workspace=None, stream=None):
    """Backward pass of the batched dot for per-vector upstream gradients g
    (2, nvec): every element i of vector v gets dx_i = g_v y_i and
    dy_i = g_v x_i (Mul22), elements of no vector zeros.  x and y are
    float-float (2, total) or binary32 (total,); the gradients are
    float-float (2, total) (None when not wanted), written into dx_out /
    dy_out when given.  workspace: uint8 device tensor of at least
    ff_dot_batched_backward_workspace_size(total) bytes (allocated per call
    when omitted)."""
    _check_ff(g, "g")
    nvec = _check_offsets(offsets, g.device)
    if g.dim() != 2 or g.shape[1] != nvec:
        raise ValueError(f"g must have shape (2, {nvec})")
    xh, xl, n = _ff_or_f32_planes(x, "x")
    yh, yl, n2 = _ff_or_f32_planes(y, "y")
    if n != n2 or x.device != g.device or y.device != g.device:
        raise ValueError("x, y and g must agree in length and device")
    dx = (ff_empty((n,), device=g.device) if dx_out is None else dx_out) if want_dx else None
    dy = (ff_empty((n,), device=g.device) if dy_out is None else dy_out) if want_dy else None
    for t, name in ((dx, "dx_out"), (dy, "dy_out")):
        if t is not None:
            _check_ff(t, name)
            if t.shape != (2, n) or t.device != g.device:
                raise ValueError(f"{name} must have shape (2, {n}) on {g.device}")
    ws = _workspace(ff_dot_batched_backward_workspace_size(n), g.device, workspace)
    gh, gl = _planes(g)
    dxh, dxl = _planes(dx) if want_dx else (_null(), _null())
    dyh, dyl = _planes(dy) if want_dy else (_null(), _null())
    with torch.cuda.device(g.device):
        check("ff_dot_batched_backward", lib.ff_dot_batched_backward(
            gh, gl, ctypes.c_void_p(offsets.data_ptr()), nvec, n, xh, xl, yh, yl, dxh, dxl, dyh,
            dyl, ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_handle(stream)))
    return dx, dy


# ---------------------------------------------------------------------- GEMM

def ff_gemm_workspace_size(M: int, N: int, K: int, algo: int = GEMM_SLICED_I8) -> int:
    """Workspace bytes of ff_gemm for this shape and algorithm."""
    return int(lib.ff_gemm_workspace_size(int(M), int(N), int(K), int(algo)))


@_on_stream
def ff_gemm(A: torch.Tensor, B: torch.Tensor, algo: int = GEMM_SLICED_I8, out=None,
            workspace=None, stream=None) -> torch.Tensor:
    """C = A B for float-float matrices A (2, M, K) and B (2, K, N).

    GEMM_SLICED_I8 (default) and GEMM_SLICED_BF16 scale each row of A and
    column of B by a power of two and cut it into 7 signed 8-bit digits, so
    an entry keeps the bits above 2^-56 of its row's (column's) largest
    entry: |C - exact| <= 2^-44 |A||B| elementwise for rows and columns of
    moderate dynamic range (normal(0,1) data at 4096^3: 2^-51.6), with the
    general bound in include/ff.h otherwise.  For rows or columns whose
    small entries matter 2^40 below their largest, use GEMM_FMA_LOOP (the
    plain Add22/Mul22 loop, about 17 times slower at 4096^3)."""
    M, K, lda = _check_matrix(A)
    K2, N, ldb = _check_matrix(B)
    if K2 != K:
        raise ValueError(f"inner dimensions differ: {K} vs {K2}")
    if A.device != B.device:
        raise ValueError("A and B on different devices")
    out = ff_empty((M, N), device=A.device) if out is None else out
    _, _, ldc = _check_matrix(out)
    if out.shape != (2, M, N):
        raise ValueError(f"out must have shape (2, {M}, {N})")
    nbytes = ff_gemm_workspace_size(M, N, K, algo)
    ws = _workspace(nbytes, A.device, workspace)
    Ah, Al = _planes(A)
    Bh, Bl = _planes(B)
    Ch, Cl = _planes(out)
    with torch.cuda.device(A.device):
        check("ff_gemm", lib.ff_gemm(M, N, K, Ah, Al, lda, Bh, Bl, ldb, Ch, Cl, ldc, int(algo),
                                     ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                     _stream_handle(stream)))
    return out


# Short names of the Python surface: float-float tensors in, float-float
# tensors out.
add, sub, mul, div = ff_add, ff_sub, ff_mul, ff_div
dot_batched, gemm, matvec = ff_dot_batched, ff_gemm, ff_matvec
from_float64, to_float64 = ff_from_f64, ff_to_f64
