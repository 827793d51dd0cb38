"""Pins for the oracle's c-transform (Definition of the c-transform, Section 2.1;
separable decomposition, Section 4.1; Lemma on c-transform properties (i))."""
import numpy as np
import pytest

from oracle import bfm as ob


def _rand(shape, seed, scale=0.3):
    return np.random.default_rng(seed).normal(scale=scale, size=shape)


@pytest.mark.parametrize("shape", [(17,), (12, 10), (9, 16), (6, 5, 4), (4, 7, 5)])
def test_separable_equals_full_minimum(shape):
    # The iterated one-dimensional minima must equal the minimum over the
    # whole grid taken in one go (non-separable brute force).
    f = _rand(shape, 1)
    a = ob.ctransform(f)
    b = ob.ctransform_bruteforce(f)
    assert np.max(np.abs(a - b)) <= 1e-13


def test_line_min_against_numpy_broadcast():
    # 1D minimum written a second way (numpy broadcast over all pairs).
    rng = np.random.default_rng(3)
    u = rng.normal(size=(5, 33))
    n = u.shape[1]
    x = (np.arange(n) + 0.5) / n
    ref = (0.5 * (x[:, None] - x[None, :]) ** 2 + u[:, None, :]).min(axis=2)
    assert np.max(np.abs(ob.line_min(u, 1) - ref)) <= 1e-14
    # the same lines stored along axis 0
    assert np.max(np.abs(ob.line_min(np.ascontiguousarray(u.T), 0).T - ref)) <= 1e-14


@pytest.mark.parametrize("shape", [(32, 24), (8, 12, 10)])
def test_ccc_equals_c_and_f_below_fcc(shape):
    # Lemma (c-transform properties) (i): f <= f^cc and f^ccc = f^c.
    f = _rand(shape, 5)
    fc = ob.ctransform(f)
    fcc = ob.ctransform(fc)
    fccc = ob.ctransform(fcc)
    assert np.all(f <= fcc + 1e-14)
    assert np.max(np.abs(fccc - fc)) <= 1e-13
    # a c-concave function is its own double transform
    assert np.max(np.abs(ob.ctransform(ob.ctransform(fcc)) - fcc)) <= 1e-13


@pytest.mark.parametrize("shape,shift", [((32, 32), (5, -3)), ((16, 24), (-2, 7)), ((12, 10, 8), (1, -2, 3))])
def test_linear_potential_closed_form(shape, shift):
    # f(y) = a.y with a a whole number of cells: the unconstrained minimiser
    # y = x + a is a grid point whenever it lies in the grid, so there
    # f^c(x) = -a.x - |a|^2 / 2 exactly.
    xs = ob.centres(shape)
    a = [s / n for s, n in zip(shift, shape)]
    f = sum(ai * xi for ai, xi in zip(a, xs)) + np.zeros(shape)
    fc = ob.ctransform(f)
    expect = -sum(ai * xi for ai, xi in zip(a, xs)) - 0.5 * sum(ai * ai for ai in a) + np.zeros(shape)
    inside = np.ones(shape, dtype=bool)
    for ax, (s, n) in enumerate(zip(shift, shape)):
        idx = np.arange(n) + s
        ok = (idx >= 0) & (idx < n)
        sh = [1] * len(shape)
        sh[ax] = n
        inside &= ok.reshape(sh)
    assert inside.sum() > 0
    assert np.max(np.abs(fc - expect)[inside]) <= 1e-14
    # outside that region the minimiser sits on the boundary: value is larger
    assert np.all(fc >= expect - 1e-14)


def test_constant_shift_and_zero():
    # (f + t)^c = f^c - t ; 0^c = 0 on the grid (x itself is a grid point).
    f = _rand((20, 20), 9)
    assert np.max(np.abs(ob.ctransform(f + 0.7) - (ob.ctransform(f) - 0.7))) <= 1e-14
    assert np.max(np.abs(ob.ctransform(np.zeros((13, 11))))) == 0.0
