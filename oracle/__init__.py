"""Float-float reference oracle -- TEST INFRASTRUCTURE ONLY.

A plain, slow CPU implementation of the float-float operators of Da Graca &
Defour, "Implementation of float-float operators on graphics hardware"
(cs/0603115), written in C (``oracle.c``) and loaded here with ctypes.

Only the test-suite, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import this package.  The HIP product library shares
no code with it and never calls it.

Every function takes and returns NumPy arrays.  Elementwise results are the
exact bits of the binary32 operation sequences of section 4.1 (Add12, Split,
Mul12, Add22, Mul22) plus Div22 (Dekker's div2); exact references (dot
products, GEMM entries) come back as ``fractions.Fraction`` values computed
without rounding.
"""
from __future__ import annotations

import contextlib
import ctypes
import os
import subprocess
from fractions import Fraction

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")

# binary32 in SSE registers, no contraction, no value-changing optimisation.
CFLAGS = [
    "-O2", "-std=c11", "-fPIC", "-shared",
    "-ffp-contract=off", "-fno-fast-math", "-frounding-math",
    "-msse2", "-mfpmath=sse",
]

ELEMENTWISE_OPS = {"add": 0, "sub": 1, "mul": 2, "mul_dekker": 3, "div": 4,
                   "add_accurate": 5, "sub_accurate": 6, "mul_accurate": 7,
                   "div_accurate": 8}


def build(force: bool = True, cc: str = "gcc", src: str = _SRC, out: str = _SO) -> str:
    """Compile ``oracle.c`` into ``liboracle.so`` (plain gcc, no GPU)."""
    if not force and os.path.exists(out) and os.path.getmtime(out) >= os.path.getmtime(src):
        return out
    tmp = out + ".tmp%d" % os.getpid()
    subprocess.run([cc, *CFLAGS, "-o", tmp, src, "-lm"], check=True)
    os.replace(tmp, out)
    return out


_F = ctypes.POINTER(ctypes.c_float)
_I64 = ctypes.POINTER(ctypes.c_int64)
_i64 = ctypes.c_int64
_int = ctypes.c_int
_D = ctypes.POINTER(ctypes.c_double)

_SIGS = {
    "oracle_abi_version": ([], _int),
    "oracle_exact_limbs": ([], _int),
    "oracle_exact_emin": ([], _int),
    "oracle_add12": ([_F, _F, _F, _F, _i64], None),
    "oracle_fast_add12": ([_F, _F, _F, _F, _i64], None),
    "oracle_split": ([_F, _F, _F, _i64], None),
    "oracle_mul12": ([_F, _F, _F, _F, _i64, _int], None),
    "oracle_add22": ([_F, _F, _F, _F, _F, _F, _i64], None),
    "oracle_sub22": ([_F, _F, _F, _F, _F, _F, _i64], None),
    "oracle_mul22": ([_F, _F, _F, _F, _F, _F, _i64, _int], None),
    "oracle_div22": ([_F, _F, _F, _F, _F, _F, _i64, _int], None),
    "oracle_add22_accurate": ([_F, _F, _F, _F, _F, _F, _i64], None),
    "oracle_sub22_accurate": ([_F, _F, _F, _F, _F, _F, _i64], None),
    "oracle_mul22_accurate": ([_F, _F, _F, _F, _F, _F, _i64], None),
    "oracle_div22_accurate": ([_F, _F, _F, _F, _F, _F, _i64], None),
    "oracle_elementwise": ([_int, _F, _F, _F, _F, _F, _F, _i64], _int),
    "oracle_dot_seq": ([_F, _F, _i64, _F], None),
    "oracle_dot_ff_seq": ([_F, _F, _i64, _F, _F, _i64, _i64, _F], None),
    "oracle_gemm_ff_seq": ([_i64, _F, _F, _i64, _F, _F, _i64, _F, _F, _i64,
                            _i64, _i64, _i64, _i64], None),
    "oracle_f32_ref": ([_int, _F, _F, _F, _F, _i64], _int),
    "oracle_sum2": ([_F, _i64, _F], None),
    "oracle_dot2": ([_F, _F, _i64, _F], None),
    "oracle_sum2_batched": ([_F, _I64, _i64, _F], None),
    "oracle_dot2_batched": ([_F, _F, _I64, _i64, _F], None),
    "oracle_dot_batched_backward": ([_F, _F, _I64, _i64, _i64, _F, _F, _F, _F, _F, _F, _F, _F],
                                    None),
    "oracle_from_f64": ([_D, _F, _F, _i64], None),
    "oracle_to_f64": ([_F, _F, _D, _i64], None),
    "oracle_horner_f32": ([_F, _int, _F, _F, _i64], None),
    "oracle_horner_comp": ([_F, _int, _F, _F, _i64], None),
    "oracle_horner_ff": ([_F, _F, _int, _F, _F, _F, _F, _i64], None),
    "oracle_ff_errors": ([_int, _F, _F, _F, _F, _F, _F, _i64, _D, _D], _int),
    "oracle_exact_dot": ([_F, _i64, _F, _i64, _i64, _I64], None),
    "oracle_exact_dot_ff": ([_F, _F, _i64, _F, _F, _i64, _i64, _I64], None),
    "oracle_exact_dot_batched": ([_F, _F, _I64, _i64, _I64], None),
    "oracle_dot_seq_batched": ([_F, _F, _I64, _i64, _F], None),
    "oracle_exact_gemm_entries": ([_i64, _F, _F, _i64, _F, _F, _i64, _I64, _I64,
                                   _i64, _I64], None),
    "oracle_exact_absgemm_entries": ([_i64, _F, _F, _i64, _F, _F, _i64, _I64,
                                      _I64, _i64, _I64], None),
}

_lib = None


def _load(path: str) -> ctypes.CDLL:
    handle = ctypes.CDLL(path)
    for name, (args, res) in _SIGS.items():
        fn = getattr(handle, name)
        fn.argtypes = args
        fn.restype = res
    return handle


def lib() -> ctypes.CDLL:
    """The loaded oracle library (built on first use if absent or stale)."""
    global _lib
    if _lib is None:
        build(force=False)
        _lib = _load(_SO)
    return _lib


@contextlib.contextmanager
def using_library(path: str):
    """Route every call to another build of ``oracle.c`` for the duration of
    the block.  The tests use it to plant a mistake in a copy of the source
    and check that the pins reject that copy."""
    global _lib
    saved = lib()
    _lib = _load(path)
    try:
        yield
    finally:
        _lib = saved


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float32)


def _p(a: np.ndarray):
    if a.dtype == np.float32:
        return a.ctypes.data_as(_F)
    if a.dtype == np.int64:
        return a.ctypes.data_as(_I64)
    if a.dtype == np.float64:
        return a.ctypes.data_as(_D)
    raise TypeError(a.dtype)


def _pair_inputs(*arrays):
    arrs = [_f32(a) for a in arrays]
    n = arrs[0].size
    for a in arrs:
        if a.size != n:
            raise ValueError("operand sizes differ")
    return arrs, n


# ---------------------------------------------------------------- primitives

def add12(a, b):
    """Add12 theorem (section 4.1): (s, r) with s = a (+) b, s + r = a + b."""
    (a, b), n = _pair_inputs(a, b)
    s, r = np.empty(n, np.float32), np.empty(n, np.float32)
    lib().oracle_add12(_p(a), _p(b), _p(s), _p(r), n)
    return s, r


def fast_add12(a, b):
    """The one-test Add12 variant (Fast2Sum), exact when |a| >= |b|."""
    (a, b), n = _pair_inputs(a, b)
    s, r = np.empty(n, np.float32), np.empty(n, np.float32)
    lib().oracle_fast_add12(_p(a), _p(b), _p(s), _p(r), n)
    return s, r


def split(a):
    """Split theorem (section 4.1) with s = 12: a = a_hi + a_lo."""
    (a,), n = _pair_inputs(a)
    hi, lo = np.empty(n, np.float32), np.empty(n, np.float32)
    lib().oracle_split(_p(a), _p(hi), _p(lo), n)
    return hi, lo


def mul12(a, b, dekker: bool = False):
    """Mul12 theorem (Dekker, section 4.1) or its FMA form: a*b = x + y."""
    (a, b), n = _pair_inputs(a, b)
    x, y = np.empty(n, np.float32), np.empty(n, np.float32)
    lib().oracle_mul12(_p(a), _p(b), _p(x), _p(y), n, int(dekker))
    return x, y


# ----------------------------------------------------------------- operators

def _binary(name, ah, al, bh, bl, *extra):
    (ah, al, bh, bl), n = _pair_inputs(ah, al, bh, bl)
    rh, rl = np.empty(n, np.float32), np.empty(n, np.float32)
    getattr(lib(), name)(_p(ah), _p(al), _p(bh), _p(bl), _p(rh), _p(rl), n, *extra)
    return rh, rl


def add22(ah, al, bh, bl):
    """Add22 theorem (section 4.1)."""
    return _binary("oracle_add22", ah, al, bh, bl)


def sub22(ah, al, bh, bl):
    """Add22 of a and -b."""
    return _binary("oracle_sub22", ah, al, bh, bl)


def add22_accurate(ah, al, bh, bl):
    """Cancellation-safe float-float sum (AccurateDWPlusDW of Joldes, Muller
    and Popescu 2017): relative error below 3u^2/(1 - 4u), u = 2^-24."""
    return _binary("oracle_add22_accurate", ah, al, bh, bl)


def sub22_accurate(ah, al, bh, bl):
    """The cancellation-safe sum of a and -b."""
    return _binary("oracle_sub22_accurate", ah, al, bh, bl)


def mul22_accurate(ah, al, bh, bl):
    """FMA-based float-float product (DWTimesDW3 of Joldes, Muller and
    Popescu, 2017): relative error at most 5u^2, u = 2^-24."""
    return _binary("oracle_mul22_accurate", ah, al, bh, bl)


def div22_accurate(ah, al, bh, bl):
    """Reciprocal-based float-float quotient (DWDivDW3 of Joldes, Muller and
    Popescu, 2017): relative error at most 9.8u^2, u = 2^-24."""
    return _binary("oracle_div22_accurate", ah, al, bh, bl)


def mul22(ah, al, bh, bl, dekker: bool = False):
    """Mul22 theorem (section 4.1), final step Add12(t1, t3)."""
    return _binary("oracle_mul22", ah, al, bh, bl, int(dekker))


def div22(ah, al, bh, bl, dekker: bool = False):
    """Div22 after Dekker's div2 (the paper defines no division)."""
    return _binary("oracle_div22", ah, al, bh, bl, int(dekker))


def elementwise(op: str, ah, al, bh, bl, out=None):
    """One operator by name ('add', 'sub', 'mul', 'mul_dekker', 'div')."""
    (ah, al, bh, bl), n = _pair_inputs(ah, al, bh, bl)
    if out is None:
        rh, rl = np.empty(n, np.float32), np.empty(n, np.float32)
    else:
        rh, rl = out
    rc = lib().oracle_elementwise(ELEMENTWISE_OPS[op], _p(ah), _p(al), _p(bh), _p(bl),
                                  _p(rh), _p(rl), n)
    if rc != 0:
        raise ValueError(op)
    return rh, rl


def sum2(x):
    """Sum2 of Ogita, Rump and Oishi (2005): returns (p, s); the result is
    the binary32 sum p (+) s."""
    (x,), n = _pair_inputs(x)
    out = np.empty(2, np.float32)
    lib().oracle_sum2(_p(x), n, _p(out))
    return out[0], out[1]


def dot2(x, y):
    """Dot2 of Ogita, Rump and Oishi (2005), FMA TwoProduct: returns (p, s);
    the result is p (+) s."""
    (x, y), n = _pair_inputs(x, y)
    out = np.empty(2, np.float32)
    lib().oracle_dot2(_p(x), _p(y), n, _p(out))
    return out[0], out[1]


def sum2_batched(x, offsets):
    (x,), _ = _pair_inputs(x)
    offs = np.ascontiguousarray(offsets, dtype=np.int64)
    out = np.empty(2 * (offs.size - 1), np.float32)
    lib().oracle_sum2_batched(_p(x), _p(offs), offs.size - 1, _p(out))
    return out[0::2].copy(), out[1::2].copy()


def dot2_batched(x, y, offsets):
    (x, y), _ = _pair_inputs(x, y)
    offs = np.ascontiguousarray(offsets, dtype=np.int64)
    out = np.empty(2 * (offs.size - 1), np.float32)
    lib().oracle_dot2_batched(_p(x), _p(y), _p(offs), offs.size - 1, _p(out))
    return out[0::2].copy(), out[1::2].copy()


def dot_batched_backward(gh, gl, offsets, xh, xl, yh, yl):
    """Gradients (dxh, dxl, dyh, dyl) of the batched float-float dot for
    upstream gradients g_v = (gh[v], gl[v]): dx_i = Mul22(g_v, y_i),
    dy_i = Mul22(g_v, x_i) for each element i of vector v, zero elsewhere."""
    (gh, gl), nvec = _pair_inputs(gh, gl)
    (xh, xl, yh, yl), n = _pair_inputs(xh, xl, yh, yl)
    offs = np.ascontiguousarray(offsets, dtype=np.int64)
    if offs.size != nvec + 1 or np.any(np.diff(offs) < 0) or offs[0] < 0 or offs[-1] > n:
        raise ValueError("offsets: nvec + 1 non-decreasing values within [0, n]")
    out = [np.empty(n, np.float32) for _ in range(4)]
    lib().oracle_dot_batched_backward(_p(gh), _p(gl), _p(offs), nvec, n, _p(xh), _p(xl),
                                      _p(yh), _p(yl), *(_p(o) for o in out))
    return tuple(out)


# --------------------------------------------------------------- conversions

def from_f64(x):
    """binary64 -> float-float: hi = fl32(x), lo = fl32(x - hi)."""
    x = np.ascontiguousarray(x, dtype=np.float64).ravel()
    hi, lo = np.empty(x.size, np.float32), np.empty(x.size, np.float32)
    lib().oracle_from_f64(_p(x), _p(hi), _p(lo), x.size)
    return hi, lo


def to_f64(hi, lo):
    """float-float -> binary64: (double) hi + (double) lo, one rounding."""
    (hi, lo), n = _pair_inputs(hi, lo)
    x = np.empty(n, np.float64)
    lib().oracle_to_f64(_p(hi), _p(lo), _p(x), n)
    return x


# ----------------------------------------------------- polynomial evaluation

def _coefficients(a):
    a = _f32(a).ravel()
    if a.size == 0:
        raise ValueError("a polynomial needs at least one coefficient")
    return a, a.size - 1


def horner_f32(a, x):
    """Horner's rule in binary32 at every point of x; a[i] multiplies x^i."""
    a, degree = _coefficients(a)
    x = _f32(x).ravel()
    y = np.empty(x.size, np.float32)
    lib().oracle_horner_f32(_p(a), degree, _p(x), _p(y), x.size)
    return y


def horner_comp(a, x):
    """Compensated Horner (Graillat, Langlois and Louvet) at every point."""
    a, degree = _coefficients(a)
    x = _f32(x).ravel()
    y = np.empty(x.size, np.float32)
    lib().oracle_horner_comp(_p(a), degree, _p(x), _p(y), x.size)
    return y


def horner_ff(ah, al, xh, xl):
    """Float-float Horner (Mul22 then Add22 per step); returns (yh, yl)."""
    (ah, al), _ = _pair_inputs(ah, al)
    ah, degree = _coefficients(ah)
    (xh, xl), n = _pair_inputs(xh, xl)
    yh, yl = np.empty(n, np.float32), np.empty(n, np.float32)
    lib().oracle_horner_ff(_p(ah), _p(al.ravel()), degree, _p(xh), _p(xl), _p(yh), _p(yl), n)
    return yh, yl


F32_REF_OPS = {"add": 0, "mul": 1, "mad": 2}


def f32_ref(op: str, a, b, c=None):
    """The binary32 reference operators of the paper's timing tables
    (section 6): 'add' a (+) b, 'mul' a (x) b, 'mad' fma(a, b, c)."""
    if c is None:
        c = np.zeros_like(_f32(a))
    (a, b, c), n = _pair_inputs(a, b, c)
    r = np.empty(n, np.float32)
    if lib().oracle_f32_ref(F32_REF_OPS[op], _p(a), _p(b), _p(c), _p(r), n) != 0:
        raise ValueError(op)
    return r


FF_ERROR_OPS = {"add22": 0, "mul22": 1, "add12": 2, "mul12": 3, "div22": 4,
                "mul22_accurate": 5, "div22_accurate": 6}


def ff_errors(op: str, ah, al, bh, bl, rh, rl):
    """Exact errors of results (rh, rl) of an operator on (ah, al), (bh, bl)
    (section 6.1): returns (rel, ratio), binary64 arrays with
    rel = |err| / |exact| and ratio = |err| / (the theorem's bound).  For
    'add12' and 'mul12' the low inputs are ignored and the bound is 0 (the
    results must be exact: ratio is +inf for any error)."""
    (ah, al, bh, bl, rh, rl), n = _pair_inputs(ah, al, bh, bl, rh, rl)
    rel, ratio = np.empty(n, np.float64), np.empty(n, np.float64)
    if lib().oracle_ff_errors(FF_ERROR_OPS[op], _p(ah), _p(al), _p(bh), _p(bl), _p(rh), _p(rl),
                              n, _p(rel), _p(ratio)) != 0:
        raise ValueError(op)
    return rel, ratio


# --------------------------------------------------------------- reductions

def dot_seq(x, y):
    """Float-float dot of FP32 vectors, Add22-accumulated in index order."""
    (x, y), n = _pair_inputs(x, y)
    out = np.empty(2, np.float32)
    lib().oracle_dot_seq(_p(x), _p(y), n, _p(out))
    return float(out[0]), float(out[1])


def dot_ff_seq(xh, xl, yh, yl):
    """Float-float dot of float-float vectors: Add22 of Mul22 terms in order."""
    (xh, xl, yh, yl), n = _pair_inputs(xh, xl, yh, yl)
    out = np.empty(2, np.float32)
    lib().oracle_dot_ff_seq(_p(xh), _p(xl), 1, _p(yh), _p(yl), 1, n, _p(out))
    return float(out[0]), float(out[1])


def dot_seq_batched(x, y, offsets):
    """Sequential float-float dots of concatenated vectors -> (hi[], lo[])."""
    (x, y), _ = _pair_inputs(x, y)
    offs = np.ascontiguousarray(offsets, dtype=np.int64)
    nvec = offs.size - 1
    out = np.empty(2 * nvec, np.float32)
    lib().oracle_dot_seq_batched(_p(x), _p(y), _p(offs), nvec, _p(out))
    return out[0::2].copy(), out[1::2].copy()


def gemm_ff_seq(Ah, Al, Bh, Bl, rows=None, cols=None):
    """Plain float-float GEMM block C[rows, cols] (Add22 over k ascending of
    Mul22 terms).  A is (M, K), B is (K, N), row-major float32."""
    Ah, Al, Bh, Bl = (_f32(m) for m in (Ah, Al, Bh, Bl))
    M, K = Ah.shape
    K2, N = Bh.shape
    if K2 != K:
        raise ValueError("inner dimensions differ")
    i0, i1 = rows if rows is not None else (0, M)
    j0, j1 = cols if cols is not None else (0, N)
    Ch = np.zeros((i1 - i0, j1 - j0), np.float32)
    Cl = np.zeros_like(Ch)
    lib().oracle_gemm_ff_seq(K, _p(Ah), _p(Al), K, _p(Bh), _p(Bl), N, _p(Ch), _p(Cl),
                             Ch.shape[1], i0, i1, j0, j1)
    return Ch, Cl


# -------------------------------------------------------- exact references

def _limb_layout():
    return lib().oracle_exact_limbs(), lib().oracle_exact_emin()


def limbs_to_fraction(limbs) -> Fraction:
    """Value of one long-accumulator result: sum_k limbs[k] 2^(32k + emin)."""
    nl, emin = _limb_layout()
    v = 0
    for k in range(nl - 1, -1, -1):
        v = (v << 32) + int(limbs[k])
    return Fraction(v, 1 << (-emin)) if emin < 0 else Fraction(v << emin)


def exact_dot(x, y) -> Fraction:
    """sum_i x_i y_i without rounding (FP32 inputs)."""
    (x, y), n = _pair_inputs(x, y)
    nl, _ = _limb_layout()
    limbs = np.empty(nl, np.int64)
    lib().oracle_exact_dot(_p(x), 1, _p(y), 1, n, _p(limbs))
    return limbs_to_fraction(limbs)


def exact_dot_ff(xh, xl, yh, yl, incx: int = 1, incy: int = 1, n: int | None = None) -> Fraction:
    """sum_i (xh_i + xl_i)(yh_i + yl_i) without rounding (strided views allowed
    through ``incx``/``incy`` on flat arrays)."""
    xh, xl, yh, yl = (_f32(v) for v in (xh, xl, yh, yl))
    if n is None:
        n = xh.size
    nl, _ = _limb_layout()
    limbs = np.empty(nl, np.int64)
    lib().oracle_exact_dot_ff(_p(xh), _p(xl), incx, _p(yh), _p(yl), incy, n, _p(limbs))
    return limbs_to_fraction(limbs)


def exact_dot_batched(x, y, offsets) -> list:
    """Exact dots of concatenated FP32 vectors (one Fraction per vector)."""
    (x, y), _ = _pair_inputs(x, y)
    offs = np.ascontiguousarray(offsets, dtype=np.int64)
    nvec = offs.size - 1
    nl, _ = _limb_layout()
    limbs = np.empty(nvec * nl, np.int64)
    lib().oracle_exact_dot_batched(_p(x), _p(y), _p(offs), nvec, _p(limbs))
    return [limbs_to_fraction(limbs[v * nl:(v + 1) * nl]) for v in range(nvec)]


def _gemm_entries(fn, Ah, Al, Bh, Bl, rows, cols):
    Ah, Al, Bh, Bl = (_f32(m) for m in (Ah, Al, Bh, Bl))
    K = Ah.shape[1]
    if Bh.shape[0] != K:
        raise ValueError("inner dimensions differ")
    r = np.ascontiguousarray(rows, dtype=np.int64)
    c = np.ascontiguousarray(cols, dtype=np.int64)
    nl, _ = _limb_layout()
    limbs = np.empty(r.size * nl, np.int64)
    fn(K, _p(Ah), _p(Al), Ah.shape[1], _p(Bh), _p(Bl), Bh.shape[1], _p(r), _p(c), r.size,
       _p(limbs))
    return [limbs_to_fraction(limbs[t * nl:(t + 1) * nl]) for t in range(r.size)]


def exact_gemm_entries(Ah, Al, Bh, Bl, rows, cols) -> list:
    """Exact C_ij = sum_k (Ah+Al)_ik (Bh+Bl)_kj for each (rows[t], cols[t])."""
    return _gemm_entries(lib().oracle_exact_gemm_entries, Ah, Al, Bh, Bl, rows, cols)


def exact_absgemm_entries(Ah, Al, Bh, Bl, rows, cols) -> list:
    """Exact (|A| |B|)_ij for each (rows[t], cols[t]): the normwise scale."""
    return _gemm_entries(lib().oracle_exact_absgemm_entries, Ah, Al, Bh, Bl, rows, cols)
