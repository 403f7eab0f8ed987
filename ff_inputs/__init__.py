"""Seeded synthetic inputs for the float-float workloads.

This module is shared by the tests, the benchmark and the smoke check; it
holds none of the float-float operators (no Add12, Split, Mul12, Add22 ...).
It only draws random numbers and converts FP64 draws into the (hi, lo) FP32
storage format: hi = fp32(x), lo = fp32(x - hi), where x - hi is exact in
FP64.

Every generator takes a seed and a torch device and returns float32 tensors;
a float-float tensor has shape (2, *shape) with plane 0 = hi, plane 1 = lo.
The same seed on the same device type always gives the same data.

Workloads (the paper measures on random vectors only; these stand in for
them):
  * ``base_ff``: x = +-2^t, t ~ U[-20, 20], fair random sign.
  * ``mixed_ff_pair``: operand pairs of the elementwise workload: 65 % base
    pairs, 25 % cancellation pairs b = -a (1 + eps), eps = +-2^V,
    V ~ U[-40, -10], and 10 % exponent-gap pairs |b| = |a| 2^(u - g),
    g integer in [24, 60], u ~ U[0, 1), random sign, a and b swapped with
    probability 1/2.
  * ``batched_dot``: 4096 vectors, lengths floor(2^U), U ~ U[6, 20]; FP32
    entries normal(0,1) * 2^k, k integer uniform in [-10, 10].
  * ``gaussian_ff``: FP64 normal(0,1) entries split into (hi, lo).
  * ``ill_conditioned_dot``: binary32 vectors whose dot product cancels to a
    prescribed condition number (the construction of Ogita, Rump and Oishi's
    test generator, 2005, section 6, written here from its description).
  * ``binomial_poly`` / ``horner_points``: the expanded (x - 1)^n, whose
    coefficients are exact binary32 integers for n <= 25, and points drawn
    uniformly around its root (the ill-conditioned test polynomial of the
    compensated Horner literature); ``random_poly``: normal(0,1)
    coefficients, binary32 or float-float.
"""
from __future__ import annotations

import torch

__all__ = [
    "split_f64", "base_ff", "mixed_ff_pair", "batched_dot", "gaussian_ff",
    "gaussian_f32", "join_f64", "random_f32", "random_ff", "scaled_normal",
    "ill_conditioned_dot", "binomial_poly", "horner_points", "random_poly",
]


def _gen(seed: int, device) -> torch.Generator:
    g = torch.Generator(device=torch.device(device))
    g.manual_seed(int(seed))
    return g


def split_f64(x: torch.Tensor) -> torch.Tensor:
    """FP64 tensor -> float-float storage (2, *shape): hi = fp32(x),
    lo = fp32(x - hi).  Data conversion only."""
    hi = x.to(torch.float32)
    lo = (x - hi.to(torch.float64)).to(torch.float32)
    return torch.stack([hi, lo])


def join_f64(ff: torch.Tensor) -> torch.Tensor:
    """Float-float storage -> FP64 value hi + lo (exact: both fit in 53 bits
    when the exponents are within 29 of each other, as generated here)."""
    return ff[0].to(torch.float64) + ff[1].to(torch.float64)


def _random_sign(n: int, g: torch.Generator, device) -> torch.Tensor:
    bits = torch.randint(0, 2, (n,), generator=g, device=device, dtype=torch.int8)
    return bits.to(torch.float64) * 2.0 - 1.0


def _base_f64(n: int, g: torch.Generator, device) -> torch.Tensor:
    t = torch.rand(n, generator=g, device=device, dtype=torch.float64) * 40.0 - 20.0
    return _random_sign(n, g, device) * torch.exp2(t)


def base_ff(n: int, seed: int, device="cpu") -> torch.Tensor:
    """n float-float values x = +-2^t, t ~ U[-20, 20] (shape (2, n))."""
    g = _gen(seed, device)
    return split_f64(_base_f64(n, g, device))


def mixed_ff_pair(n: int, seed: int, device="cpu", p_cancel: float = 0.25,
                  p_gap: float = 0.10):
    """Operand pair (a, b), each (2, n), for the elementwise workload.

    Categories are drawn per index from one uniform: [0, p_cancel) are
    cancellation pairs, [p_cancel, p_cancel + p_gap) exponent-gap pairs,
    the rest independent base pairs.  Returns (a, b, category) with
    category 0 = base, 1 = cancellation, 2 = gap (int8).
    """
    g = _gen(seed, device)
    xa = _base_f64(n, g, device)
    xb = _base_f64(n, g, device)
    cat_u = torch.rand(n, generator=g, device=device, dtype=torch.float64)
    # cancellation: b = -a (1 + eps), eps = +-2^V, V ~ U[-40, -10]
    v = torch.rand(n, generator=g, device=device, dtype=torch.float64) * 30.0 - 40.0
    eps = _random_sign(n, g, device) * torch.exp2(v)
    xb_cancel = -xa * (1.0 + eps)
    # gap: |b| = |a| 2^(u - gap), random sign, swap with probability 1/2
    gap = torch.randint(24, 61, (n,), generator=g, device=device).to(torch.float64)
    u = torch.rand(n, generator=g, device=device, dtype=torch.float64)
    xb_gap = _random_sign(n, g, device) * xa.abs() * torch.exp2(u - gap)
    swap = torch.rand(n, generator=g, device=device, dtype=torch.float64) < 0.5

    category = torch.zeros(n, dtype=torch.int8, device=device)
    is_cancel = cat_u < p_cancel
    is_gap = (cat_u >= p_cancel) & (cat_u < p_cancel + p_gap)
    category[is_cancel] = 1
    category[is_gap] = 2

    xb = torch.where(is_cancel, xb_cancel, xb)
    xb = torch.where(is_gap, xb_gap, xb)
    do_swap = is_gap & swap
    xa2 = torch.where(do_swap, xb, xa)
    xb2 = torch.where(do_swap, xa, xb)
    return split_f64(xa2), split_f64(xb2), category


def batched_dot(seed: int, device="cpu", nvec: int = 4096, log2_min: float = 6.0,
                log2_max: float = 20.0, max_total: int | None = None):
    """Uneven FP32 dot-product batch: (x, y, offsets).

    Lengths L_v = floor(2^U), U ~ U[log2_min, log2_max], clamped to
    [2^log2_min, 2^log2_max]; entries normal(0,1) * 2^k, k uniform integer in
    [-10, 10] (the scaling by 2^k is exact).  ``offsets`` is int64 [nvec + 1]
    on the same device.  ``max_total`` scales lengths down proportionally (for
    oracle-sized cases) while keeping every length >= 1.
    """
    g = _gen(seed, device)
    u = torch.rand(nvec, generator=g, device=device, dtype=torch.float64)
    u = u * (log2_max - log2_min) + log2_min
    lengths = torch.floor(torch.exp2(u)).to(torch.int64)
    lengths = lengths.clamp(int(2 ** log2_min), int(2 ** log2_max))
    if max_total is not None and int(lengths.sum()) > max_total:
        scale = max_total / float(lengths.sum())
        lengths = torch.clamp((lengths.to(torch.float64) * scale).floor().to(torch.int64), min=1)
    offsets = torch.zeros(nvec + 1, dtype=torch.int64, device=device)
    offsets[1:] = torch.cumsum(lengths, 0)
    total = int(offsets[-1])
    x = _scaled_normal(total, g, device)
    y = _scaled_normal(total, g, device)
    return x, y, offsets


def _scaled_normal(n: int, g: torch.Generator, device) -> torch.Tensor:
    z = torch.randn(n, generator=g, device=device, dtype=torch.float32)
    k = torch.randint(-10, 11, (n,), generator=g, device=device, dtype=torch.int32)
    # 2^k built from its bit pattern (biased exponent, zero significand), so
    # the scaling is exact whatever the device's exp2/pow accuracy.
    scale = ((k + 127) << 23).view(torch.float32)
    return z * scale


def scaled_normal(n: int, seed: int, device="cpu") -> torch.Tensor:
    """n binary32 entries normal(0,1) * 2^k, k uniform integer in [-10, 10]
    (the entry distribution of the batched dot workload)."""
    return _scaled_normal(n, _gen(seed, device), device)


def gaussian_ff(shape, seed: int, device="cpu") -> torch.Tensor:
    """Float-float tensor (2, *shape) from FP64 normal(0,1) draws."""
    g = _gen(seed, device)
    x = torch.randn(tuple(shape), generator=g, device=device, dtype=torch.float64)
    return split_f64(x)


def gaussian_f32(shape, seed: int, device="cpu") -> torch.Tensor:
    """FP32 normal(0,1) tensor."""
    g = _gen(seed, device)
    return torch.randn(tuple(shape), generator=g, device=device, dtype=torch.float32)


def _from_fields(sign: torch.Tensor, exp: torch.Tensor, frac: torch.Tensor) -> torch.Tensor:
    """binary32 values from sign bit, unbiased exponent (normal range) and
    23-bit fraction field, assembled as bit patterns."""
    bits = (sign.to(torch.int32) << 31) | ((exp.to(torch.int32) + 127) << 23) | frac.to(torch.int32)
    return bits.view(torch.float32)


def random_f32(n: int, seed: int, emin: int = -40, emax: int = 40, device="cpu") -> torch.Tensor:
    """binary32 values with random sign, exponent uniform in [emin, emax]
    (normal range) and uniformly random 23-bit fraction field."""
    g = _gen(seed, device)
    sign = torch.randint(0, 2, (n,), generator=g, device=device, dtype=torch.int32)
    exp = torch.randint(emin, emax + 1, (n,), generator=g, device=device, dtype=torch.int32)
    frac = torch.randint(0, 1 << 23, (n,), generator=g, device=device, dtype=torch.int32)
    return _from_fields(sign, exp, frac)


def random_ff(n: int, seed: int, emin: int = -40, emax: int = 40, max_gap: int = 6,
              p_zero_lo: float = 0.05, device="cpu") -> torch.Tensor:
    """Normalised float-float pairs (2, n): hi as in ``random_f32``; lo has a
    random sign and fraction and exponent E(hi) - 25 - g, g uniform in
    [0, max_gap], so |lo| < ulp(hi)/2; a fraction p_zero_lo of lo words is 0."""
    g = _gen(seed, device)
    sign = torch.randint(0, 2, (n,), generator=g, device=device, dtype=torch.int32)
    exp = torch.randint(emin, emax + 1, (n,), generator=g, device=device, dtype=torch.int32)
    frac = torch.randint(0, 1 << 23, (n,), generator=g, device=device, dtype=torch.int32)
    hi = _from_fields(sign, exp, frac)
    lsign = torch.randint(0, 2, (n,), generator=g, device=device, dtype=torch.int32)
    gap = torch.randint(0, max_gap + 1, (n,), generator=g, device=device, dtype=torch.int32)
    lfrac = torch.randint(0, 1 << 23, (n,), generator=g, device=device, dtype=torch.int32)
    lo = _from_fields(lsign, exp - 25 - gap, lfrac)
    zero = torch.rand(n, generator=g, device=device) < p_zero_lo
    lo = torch.where(zero, torch.zeros_like(lo), lo)
    return torch.stack([hi, lo])


def ill_conditioned_dot(n: int, seed: int, log2_cond: float = 40.0, device="cpu"):
    """binary32 x, y of length n (n >= 6) whose dot product has condition
    number 2 sum|x_i y_i| / |x.y| near 2^log2_cond.  The first half holds
    random entries whose exponents spread over [0, log2_cond / 2]; in the
    second half, with exponents falling from log2_cond / 2 to 0, each y_i
    is chosen so that x_i y_i cancels the running sum (kept in FP64) down to
    a random value of the current magnitude.  The entries are then shuffled.
    Data generation only: the exact dot product and its condition number
    are measured by the caller."""
    if n < 6:
        raise ValueError("n >= 6")
    g = _gen(seed, "cpu")
    half = n // 2
    b = log2_cond / 2.0
    e1 = torch.round(torch.rand(half, generator=g, dtype=torch.float64) * b)
    e1[0], e1[-1] = round(b), 0.0
    x1 = ((2 * torch.rand(half, generator=g, dtype=torch.float64) - 1) * torch.exp2(e1)).float()
    y1 = ((2 * torch.rand(half, generator=g, dtype=torch.float64) - 1) * torch.exp2(e1)).float()
    rest = n - half
    e2 = torch.round(torch.linspace(b, 0.0, rest, dtype=torch.float64))
    x2 = ((2 * torch.rand(rest, generator=g, dtype=torch.float64) - 1) * torch.exp2(e2)).float()
    target = (2 * torch.rand(rest, generator=g, dtype=torch.float64) - 1) * torch.exp2(e2)
    y2 = torch.empty(rest, dtype=torch.float32)
    run = float((x1.double() * y1.double()).sum())
    for i in range(rest):
        xi = float(x2[i])
        yi = torch.tensor((float(target[i]) - run) / xi, dtype=torch.float64).float()
        y2[i] = yi
        run += xi * float(yi)
    perm = torch.randperm(n, generator=g)
    x = torch.cat([x1, x2])[perm].contiguous()
    y = torch.cat([y1, y2])[perm].contiguous()
    return x.to(device), y.to(device)


def binomial_poly(n: int) -> torch.Tensor:
    """Coefficients, ascending, of the expanded (x - 1)^n: a_i = C(n, i)
    (-1)^(n - i).  Every one is an integer below 2^24, so binary32 holds it
    exactly, for n <= 25."""
    import math

    if not 0 <= n <= 25:
        raise ValueError("0 <= n <= 25")
    return torch.tensor([math.comb(n, i) * (-1) ** (n - i) for i in range(n + 1)],
                        dtype=torch.float32)


def horner_points(n: int, seed: int, lo: float, hi: float, device="cpu") -> torch.Tensor:
    """n binary32 points drawn uniformly from [lo, hi] (FP64 draws rounded)."""
    g = _gen(seed, device)
    u = torch.rand(n, generator=g, device=device, dtype=torch.float64)
    return (lo + (hi - lo) * u).float()


def random_poly(degree: int, seed: int, ff: bool = False) -> torch.Tensor:
    """degree + 1 normal(0,1) coefficients: binary32 (shape (degree + 1,)),
    or FP64 draws split into float-float (shape (2, degree + 1))."""
    g = _gen(seed, "cpu")
    a = torch.randn(degree + 1, generator=g, dtype=torch.float64)
    return split_f64(a) if ff else a.float()
