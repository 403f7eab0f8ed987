"""The C ABI (include/ff.h) on the host: the library loads, exports every
declared entry point, and rejects invalid arguments before any HIP call.

No test here launches work: the validation paths return before touching the
HIP runtime, so fake host addresses are safe.
"""
import ctypes
import os
import re
import subprocess

import pytest

import paper_cs_0603115_amd as ff
from paper_cs_0603115_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER_DIR = os.path.join(ROOT, "include")

ERR_NULL, ERR_SIZE, ERR_ALIGN, ERR_WS, ERR_UNSUP, ERR_HIP, ERR_ARG = 1, 2, 3, 4, 5, 6, 7


def declared_functions():
    names = []
    for fname in sorted(os.listdir(HEADER_DIR)):
        if not fname.endswith(".h"):
            continue
        text = open(os.path.join(HEADER_DIR, fname)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        text = "\n".join(l for l in text.splitlines() if not l.lstrip().startswith("#"))
        names += re.findall(r"\b(ff_\w+)\s*\([^;{]*\)\s*;", text)
    return names


def exported_symbols():
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    return {line.split()[-1] for line in out.splitlines() if line.strip()}


def test_header_declares_entry_points():
    names = declared_functions()
    assert len(names) == len(set(names))
    for required in ("ff_add", "ff_sub", "ff_mul", "ff_mul_dekker", "ff_div"):
        assert required in names


def test_every_declared_symbol_is_exported_and_bound():
    exported = exported_symbols()
    for name in declared_functions():
        assert name in exported, f"{name} declared in include/ but not exported"
        assert name in _lib.SIGNATURES, f"{name} missing from the Python binding"
        assert hasattr(_lib.lib, name)
    for name in _lib.SIGNATURES:
        assert name in declared_functions(), f"{name} bound but not declared"


def test_version_and_build_info():
    assert ff.lib.ff_abi_version() == 1
    info = ff.build_info()
    for token in ("gfx950", "fp-contract=off", "f32-denormals=preserve",
                  "f32-division=correctly-rounded"):
        assert token in info


def test_status_strings():
    for code, name in _lib.STATUS_NAMES.items():
        assert ff.lib.ff_status_str(code).decode() == name
    assert ff.lib.ff_status_str(99).decode() == "FF_ERR_UNKNOWN"
    assert ff.lib.ff_last_error().decode() == ""


EW = ["ff_add", "ff_sub", "ff_mul", "ff_mul_dekker", "ff_div", "ff_add_accurate", "ff_sub_accurate",
      "ff_mul_accurate", "ff_div_accurate"]


@pytest.mark.parametrize("name", EW)
def test_elementwise_validation(name):
    fn = getattr(ff.lib, name)
    p = [4096 * (k + 1) for k in range(6)]          # fake 16-byte aligned addresses
    assert fn(*p, -1, None) == ERR_SIZE
    assert fn(*p, 0, None) == 0                     # no-op, nothing enqueued
    assert fn(None, None, None, None, None, None, 0, None) == 0
    for k in range(6):
        q = list(p)
        q[k] = None
        assert fn(*q, 10, None) == ERR_NULL
        q = list(p)
        q[k] = p[k] + 2                             # not 4-byte aligned
        assert fn(*q, 10, None) == ERR_ALIGN


@pytest.mark.parametrize("name,nptr", [("ff_add12", 4), ("ff_mul12", 4), ("ff_mul12_dekker", 4),
                                       ("ff_f32_add", 3), ("ff_f32_mul", 3), ("ff_f32_mad", 4)])
def test_stream_operator_validation(name, nptr):
    fn = getattr(ff.lib, name)
    p = [4096 * (k + 1) for k in range(nptr)]
    assert fn(*p, -1, None) == ERR_SIZE
    assert fn(*p, 0, None) == 0
    assert fn(*([None] * nptr), 0, None) == 0
    for k in range(nptr):
        q = list(p)
        q[k] = None
        assert fn(*q, 10, None) == ERR_NULL
        q = list(p)
        q[k] = p[k] + 2
        assert fn(*q, 10, None) == ERR_ALIGN


@pytest.mark.parametrize("name", ["ff_horner_f32", "ff_horner_comp"])
def test_horner_validation(name):
    fn = getattr(ff.lib, name)
    c, x, y = 4096, 8192, 12288
    assert fn(c, -1, x, y, 10, None) == ERR_SIZE
    assert fn(c, 3, x, y, -1, None) == ERR_SIZE
    assert fn(None, 3, None, None, 0, None) == 0    # n = 0: no-op
    for q in ((None, x, y), (c, None, y), (c, x, None)):
        assert fn(q[0], 3, q[1], q[2], 10, None) == ERR_NULL
    for q in ((c + 2, x, y), (c, x + 2, y), (c, x, y + 2)):
        assert fn(q[0], 3, q[1], q[2], 10, None) == ERR_ALIGN


def test_horner_ff_validation():
    fn = ff.lib.ff_horner_ff
    p = [4096 * (k + 1) for k in range(6)]          # ch, cl, xh, xl, yh, yl
    call = lambda q, degree=3, n=10: fn(q[0], q[1], degree, q[2], q[3], q[4], q[5], n, None)
    assert call(p, degree=-2) == ERR_SIZE
    assert call(p, n=-1) == ERR_SIZE
    assert call([None] * 6, n=0) == 0
    for k in (0, 2, 4, 5):                          # coefficient and point low words may be null
        q = list(p)
        q[k] = None
        assert call(q) == ERR_NULL
    for k in range(6):
        q = list(p)
        q[k] = p[k] + 2
        assert call(q) == ERR_ALIGN


@pytest.mark.parametrize("name", ["ff_from_f64", "ff_to_f64"])
def test_conversion_validation(name):
    fn = getattr(ff.lib, name)
    f64 = 4096
    f32 = (8192, 12288)
    call = (lambda d, h, l, n: fn(d, h, l, n, None)) if name == "ff_from_f64" else \
        (lambda d, h, l, n: fn(h, l, d, n, None))
    assert call(f64, *f32, -1) == ERR_SIZE
    assert call(None, None, None, 0) == 0
    assert call(None, *f32, 5) == ERR_NULL
    assert call(f64, None, f32[1], 5) == ERR_NULL
    assert call(f64 + 4, *f32, 5) == ERR_ALIGN          # binary64 plane needs 8 bytes
    assert call(f64, f32[0] + 2, f32[1], 5) == ERR_ALIGN


def test_dot_batched_backward_validation():
    fn = ff.lib.ff_dot_batched_backward
    g, o = (4096, 8192), 12288
    xs, ys = (16384, 20480), (24576, 28672)
    d = (32768, 36864, 40960, 45056)
    ws = 49152
    call = lambda gg=g, off=o, nvec=3, total=100, x=xs, y=ys, out=d, w=ws, wb=4096: fn(
        gg[0], gg[1], off, nvec, total, x[0], x[1], y[0], y[1], *out, w, wb, None)
    size = ff.lib.ff_dot_batched_backward_workspace_size
    assert size(0) == 0 and size(-5) == 0
    assert size(1) == 16 and size(256) == 16 and size(257) == 32
    assert size(438907317) == 16 * -(-438907317 // 256)
    assert call(nvec=-1) == ERR_SIZE
    assert call(total=-1) == ERR_SIZE
    assert call(total=0) == 0
    assert call(out=(None, None, None, None)) == 0          # nothing wanted: no-op
    assert call(out=(d[0], None, d[2], d[3])) == ERR_NULL   # half an output pair
    assert call(off=None) == ERR_NULL
    assert call(gg=(None, g[1])) == ERR_NULL
    assert call(y=(None, ys[1])) == ERR_NULL                # dx needs y
    assert call(off=o + 4) == ERR_ALIGN                     # offsets need 8 bytes
    assert call(x=(xs[0] + 2, xs[1])) == ERR_ALIGN
    assert call(w=None) == ERR_WS
    assert call(wb=15) == ERR_WS                     # 100 elements: one 16-byte record
    assert call(total=257, wb=16) == ERR_WS          # two records
    assert call(w=ws + 8) == ERR_ALIGN                      # records need 16 bytes
    assert call(total=0, w=None) == 0                       # no-op reads no workspace
    assert call(out=(None, None, None, None), w=None) == 0


def test_copy_validation():
    assert ff.lib.ff_copy(4096, 8192, -3, None) == ERR_SIZE
    assert ff.lib.ff_copy(4096, 8192, 0, None) == 0
    assert ff.lib.ff_copy(None, 8192, 4, None) == ERR_NULL
    assert ff.lib.ff_copy(4097, 8192, 4, None) == ERR_ALIGN


def test_python_binding_rejects_bad_tensors():
    import torch
    a = torch.zeros(2, 8)
    with pytest.raises(ValueError):
        ff.ff_add(a, a)                              # CPU tensor: the library is GPU-only
    with pytest.raises(ValueError):
        ff.ff_add(torch.zeros(3, 8), torch.zeros(3, 8))
    with pytest.raises(TypeError):
        ff.ff_add(a.double(), a.double())


def test_ff_error_carries_status():
    with pytest.raises(ff.FFError) as err:
        _lib.check("ff_add", ERR_ALIGN)
    assert err.value.status == ERR_ALIGN and "FF_ERR_ALIGN" in str(err.value)


def test_dot_workspace_size():
    size = ff.ff_dot_batched_workspace_size
    assert size(0, 0) > 0 or size(0, 0) == 0
    assert size(1 << 20, 10) > 0
    assert size(-1, 10) == 0 and size(10, -1) == 0
    assert size(100, 3, (0, 0, 0, 3)) == 0          # unroll: a power of two up to 32
    assert size(100, 3, (0, 0, 0, 64)) == 0
    assert size(100, 3, (0, 60, 0, 0)) == 0         # chunk must be block * unroll
    assert size(100, 3, (256, 1024, 0, 8)) == 0
    assert size(100, 3, (96, 0, 0, 0)) == 0         # block 64, 128, 256 or 512
    assert size(100, 3, (256, 0, 7, 0)) == 0        # grid reserved: zero
    assert size(100, 3, (0, 1024, 0, 0)) > 0        # chunk alone sets unroll = chunk / block
    # grows with the chunk count (total / chunk + nvec partials)
    assert size(1 << 24, 4, (64, 256, 0, 4)) > size(1 << 24, 4, (512, 16384, 0, 32))


@pytest.mark.parametrize("name", ["ff_dot_batched", "ff_dot_ff_batched", "ff_dot2_batched",
                                  "ff_sum_batched", "ff_sum2_batched"])
def test_dot_validation(name):
    fn = getattr(ff.lib, name)
    nplanes = {"ff_dot_batched": 2, "ff_dot2_batched": 2, "ff_dot_ff_batched": 4,
               "ff_sum_batched": 1, "ff_sum2_batched": 1}[name]
    planes = [4096 * (k + 1) for k in range(nplanes)]
    offs, oh, ol, ws = 1 << 20, 2 << 20, 3 << 20, 4 << 20
    need = ff.ff_dot_batched_workspace_size(1000, 8)

    def call(planes=planes, offs=offs, nvec=8, total=1000, cfg=None, ws=ws, ws_bytes=need,
             oh=oh, ol=ol):
        cfgp = None if cfg is None else ctypes.byref(_lib.DotCfg(*cfg))
        return fn(*planes, offs, nvec, total, cfgp, ws, ws_bytes, oh, ol, None)

    assert call(nvec=-1) == ERR_SIZE
    assert call(total=-5) == ERR_SIZE
    assert call(nvec=0) == 0                           # nothing to do
    assert call(cfg=(0, 0, 0, 3)) == ERR_ARG
    assert call(cfg=(1024, 0, 0, 0)) == ERR_ARG
    assert call(ws_bytes=need - 1) == ERR_WS
    assert call(ws=None) == ERR_NULL
    assert call(offs=None) == ERR_NULL
    assert call(oh=None) == ERR_NULL
    p = list(planes)
    p[0] = None
    assert call(planes=p) == ERR_NULL
    p = list(planes)
    p[-1] = planes[-1] + 1
    assert call(planes=p) == ERR_ALIGN
    assert call(offs=offs + 4) == ERR_ALIGN
    assert call(ws=ws + 64) == ERR_ALIGN


def test_dot_noalloc_validation():
    """The allocation-free batched dot checks its arguments, and its static
    scratch limit, before any HIP call."""
    fn = ff.lib.ff_dot_batched_noalloc
    x, y, offs, oh, ol = 4096, 8192, 1 << 20, 2 << 20, 3 << 20

    def call(x=x, y=y, offs=offs, nvec=8, total=1000, cfg=None, oh=oh, ol=ol):
        cfgp = None if cfg is None else ctypes.byref(_lib.DotCfg(*cfg))
        return fn(x, y, offs, nvec, total, cfgp, oh, ol, None)

    assert call(nvec=-1) == ERR_SIZE
    assert call(total=-5) == ERR_SIZE
    assert call(nvec=0) == 0                           # nothing to do
    assert call(cfg=(0, 0, 0, 3)) == ERR_ARG
    assert call(x=None) == ERR_NULL
    assert call(offs=None) == ERR_NULL
    assert call(ol=None) == ERR_NULL
    assert call(y=y + 2) == ERR_ALIGN
    assert call(offs=offs + 4) == ERR_ALIGN
    # the batch must fit the static scratch: 16 MiB; 4096 vectors of up to
    # 5.68e9 elements at the default shape (8192 elements per chunk), half as
    # many at 4096 elements per chunk
    limit = 16 << 20
    assert ff.ff_dot_batched_workspace_size(5_681_717_247, 4096) <= limit
    assert ff.ff_dot_batched_workspace_size(5_681_717_248, 4096) > limit
    shape = (256, 4096, 0, 16)
    assert ff.ff_dot_batched_workspace_size(2_840_858_623, 4096, shape) <= limit
    assert ff.ff_dot_batched_workspace_size(2_840_858_623 + 4096, 4096, shape) > limit
    assert call(nvec=4096, total=(1 << 14) * (1 << 20)) == ERR_WS
    assert call(nvec=1_000_000, total=1000) == ERR_WS   # too many vectors
    assert call(nvec=8, total=1 << 40, cfg=(64, 256, 0, 4)) == ERR_WS
    assert call(cfg=(256, 0, 3, 0)) == ERR_ARG


def test_matvec_validation():
    mv = ff.lib.ff_matvec
    A = [4096, 8192]
    x = [12288, 16384]
    y = [20480, 24576]
    assert mv(-1, 4, *A, 4, *x, *y, 0, None) == ERR_SIZE
    assert mv(4, 4, *A, 3, *x, *y, 0, None) == ERR_SIZE       # lda < N
    assert mv(4, 4, *A, 4, *x, *y, 2, None) == ERR_ARG        # unknown algo
    assert mv(0, 4, *A, 4, *x, *y, 0, None) == 0              # nothing to do
    assert mv(4, 4, None, A[1], 4, *x, *y, 0, None) == ERR_NULL
    assert mv(4, 4, *A, 4, *x, y[0] + 2, y[1], 0, None) == ERR_ALIGN
    bw = ff.lib.ff_matvec_backward
    g = [28672, 32768]
    dA = [36864, 40960]
    dx = [45056, 49152]
    # partial sums: one float2 per 128-row band and column
    assert ff.lib.ff_matvec_backward_workspace_size(300, 4, 0) == 3 * 4 * 8
    need = ff.lib.ff_matvec_backward_workspace_size(100, 4, 0)
    assert need == 1 * 4 * 8
    assert ff.lib.ff_matvec_backward_workspace_size(100, 4, 1) == 0
    ws = 1 << 20
    assert bw(100, 4, *A, 4, *x, *g, *dA, 4, *dx, 0, ws, need - 1, None) == ERR_WS
    assert bw(100, 4, *A, 4, *x, *g, *dA, 3, *dx, 0, ws, need, None) == ERR_SIZE
    assert bw(100, 4, *A, 4, *x, *g, dA[0], None, 4, *dx, 0, ws, need, None) == ERR_NULL
    assert bw(100, 4, *A, 4, *x, *g, None, None, 4, None, None, 0, ws, need, None) == 0
    assert bw(100, 4, *A, 4, *x, *g, *dA, 4, *dx, 5, ws, need, None) == ERR_ARG
    db = ff.lib.ff_dot_backward
    assert db(*g, *x, *y, *dx, *dA, -1, None) == ERR_SIZE
    assert db(*g, *x, *y, *dx, *dA, 0, None) == 0
    assert db(None, g[1], *x, *y, *dx, *dA, 8, None) == ERR_NULL
    assert db(*g, *x, *y, dx[0], None, *dA, 8, None) == ERR_NULL


def test_sum_and_autotune_validation():
    assert ff.lib.ff_sum_batched(4096, 8192, -1, 10, None, 1 << 20, 1 << 16, 1 << 21, 1 << 22,
                                 None) == ERR_SIZE
    assert ff.lib.ff_sum_ff_batched(4096, 4098, 8192, 2, 10, None, 1 << 20, 1 << 16, 1 << 21,
                                    1 << 22, None) == ERR_ALIGN
    best = _lib.DotCfg()
    ms = ctypes.c_float()
    assert ff.lib.ff_dot_batched_autotune(4096, 8192, 12288, 4, 100, 1 << 20, 1 << 16, 1 << 21,
                                          1 << 22, 0, None, ctypes.byref(best),
                                          ctypes.byref(ms)) == ERR_ARG
    assert ff.lib.ff_dot_batched_autotune(4096, 8192, 12288, 4, 100, 1 << 20, 1 << 16, 1 << 21,
                                          1 << 22, 3, None, None, ctypes.byref(ms)) == ERR_NULL


def test_gemm_validation_and_workspace():
    g = ff.lib.ff_gemm
    size = ff.lib.ff_gemm_workspace_size
    assert size(64, 64, 64, 0) == 0                       # FMA loop needs none
    w8, w16 = size(100, 70, 333, 2), size(100, 70, 333, 1)
    assert w8 > 0 and w16 > w8
    # int8 digit planes: 7 slices x (rows and columns padded to 128) x K
    # padded to the 32-byte stage
    assert w8 >= 7 * (128 + 128) * 352
    assert size(-1, 4, 4, 2) == 0 and size(4, 4, 4, 9) == 0
    P = [4096 * (k + 1) for k in range(6)]
    ws = 1 << 24
    assert g(-1, 4, 4, P[0], P[1], 4, P[2], P[3], 4, P[4], P[5], 4, 0, None, 0, None) == ERR_SIZE
    assert g(4, 4, 4, P[0], P[1], 3, P[2], P[3], 4, P[4], P[5], 4, 0, None, 0, None) == ERR_SIZE
    assert g(4, 4, 4, P[0], P[1], 4, P[2], P[3], 4, P[4], P[5], 3, 0, None, 0, None) == ERR_SIZE
    assert g(4, 4, 4, P[0], P[1], 4, P[2], P[3], 4, P[4], P[5], 4, 7, None, 0, None) == ERR_ARG
    assert g(0, 4, 4, P[0], P[1], 4, P[2], P[3], 4, P[4], P[5], 4, 2, None, 0, None) == 0
    assert g(4, 4, 4, None, P[1], 4, P[2], P[3], 4, P[4], P[5], 4, 0, None, 0, None) == ERR_NULL
    assert g(4, 4, 4, P[0], P[1], 4, P[2], P[3] + 1, 4, P[4], P[5], 4, 0, None, 0, None) == ERR_ALIGN
    need = size(4, 4, 4, 2)
    assert g(4, 4, 4, *P[:2], 4, *P[2:4], 4, *P[4:], 4, 2, None, need, None) == ERR_NULL
    assert g(4, 4, 4, *P[:2], 4, *P[2:4], 4, *P[4:], 4, 2, ws, need - 1, None) == ERR_WS
    assert g(4, 4, 4, *P[:2], 4, *P[2:4], 4, *P[4:], 4, 2, ws + 16, need, None) == ERR_ALIGN


def test_import_fails_loudly_without_the_library(tmp_path):
    # a copy of the package without libff.so: the import itself must fail
    # (no CPU fallback exists)
    import shutil
    import sys
    src = os.path.dirname(ff.__file__)
    dst = tmp_path / "paper_cs_0603115_amd"
    dst.mkdir()
    for name in os.listdir(src):
        if name.endswith(".py"):
            shutil.copy(os.path.join(src, name), dst / name)
    r = subprocess.run([sys.executable, "-c", "import paper_cs_0603115_amd"], cwd=tmp_path,
                       env={**os.environ, "PYTHONPATH": str(tmp_path)}, capture_output=True,
                       text=True, timeout=300)
    assert r.returncode != 0
    assert "libff.so not found" in r.stderr


def test_ff_empty_planes_start_4kib_apart():
    """ff_empty / ff_zeros: two contiguous planes whose starts differ by a
    multiple of 4 KiB, so both share the allocation's alignment (host
    tensors are enough to check the layout)."""
    import torch
    for shape in [(), (0,), (1,), (63,), (1025,), (3, 7), (438907317 // 4096,)]:
        for make in (ff.ff_empty, ff.ff_zeros):
            t = make(shape, device="cpu")
            assert t.shape == (2, *shape)
            assert t.dtype == torch.float32
            assert t[0].is_contiguous() and t[1].is_contiguous()
            assert (t[1].data_ptr() - t[0].data_ptr()) % 4096 == 0
            assert t.stride(0) >= max(t[0].numel(), 1)
    z = ff.ff_zeros((5, 3), device="cpu")
    assert not z.any()
