"""Pins of the oracle's backward pass of the batched float-float dot.

s_v = sum over vector v of x_i y_i, so ds_v/dx_i = y_i and ds_v/dy_i = x_i
for the elements i of vector v (and 0 elsewhere).  With upstream gradients
g_v the gradients are dx_i = g_v y_i and dy_i = g_v x_i, formed by Mul22.

* power-of-two gradients g_v = 2^k_v: Mul22 by a power of two is exact, so
  dx_i = 2^k_v (yh_i, yl_i) bit for bit -- which also pins which vector each
  element belongs to; elements before the first vector, after the last and
  in empty vectors get zeros;
* general float-float gradients: each result within the Mul22 theorem's
  2^-44 of the exact product g_v y_i (exact Fraction arithmetic).
"""
from fractions import Fraction

import numpy as np
import pytest

import ff_inputs as fi
import oracle
from fpexact import ff_value, same_bits


def _batch(seed):
    x = fi.random_ff(3000, seed, -20, 20).numpy()
    y = fi.random_ff(3000, seed + 1, -20, 20).numpy()
    # a leading gap, empty vectors, a trailing gap
    offsets = np.array([7, 7, 100, 101, 1500, 1500, 2990], dtype=np.int64)
    return x, y, offsets


def test_power_of_two_gradients_are_exact_and_segment_correctly():
    x, y, offs = _batch(4001)
    nvec = offs.size - 1
    k = np.arange(nvec) - 3
    gh = np.ldexp(np.ones(nvec), k).astype(np.float32)
    gl = np.zeros(nvec, np.float32)
    dxh, dxl, dyh, dyl = oracle.dot_batched_backward(gh, gl, offs, x[0], x[1], y[0], y[1])
    owner = np.full(x.shape[1], -1)
    for v in range(nvec):
        owner[offs[v]:offs[v + 1]] = v
    inside = owner >= 0
    scale = np.where(inside, np.ldexp(1.0, np.where(inside, owner - 3, 0)), 0.0).astype(np.float32)
    assert same_bits(dxh[inside], y[0][inside] * scale[inside])
    assert same_bits(dxl[inside], y[1][inside] * scale[inside])
    assert same_bits(dyh[inside], x[0][inside] * scale[inside])
    assert same_bits(dyl[inside], x[1][inside] * scale[inside])
    for arr in (dxh, dxl, dyh, dyl):
        assert np.all(arr[~inside].view(np.uint32) == 0)


def test_general_gradients_within_the_mul22_bound():
    x, y, offs = _batch(4011)
    nvec = offs.size - 1
    g = fi.random_ff(nvec, 4013, -5, 5).numpy()
    dxh, dxl, dyh, dyl = oracle.dot_batched_backward(g[0], g[1], offs, x[0], x[1], y[0], y[1])
    for v in range(nvec):
        gv = ff_value(g[0][v], g[1][v])
        for i in range(offs[v], offs[v + 1], 3):
            for (dh, dl, src) in ((dxh, dxl, y), (dyh, dyl, x)):
                exact = gv * ff_value(src[0][i], src[1][i])
                assert abs(ff_value(dh[i], dl[i]) - exact) <= abs(exact) / 2 ** 44, (v, i)


def test_rejects_bad_offsets():
    x, y, _ = _batch(4021)
    g = np.ones(2, np.float32)
    with pytest.raises(ValueError):
        oracle.dot_batched_backward(g, g, np.array([0, 10, 5]), x[0], x[1], y[0], y[1])
