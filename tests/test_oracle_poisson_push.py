"""Pins for the oracle's Neumann Poisson solve (H^1-gradient lemma; Laplace
inversion of Section 4.3), map and pushforward (Section 2.1 test-function
definition of T#mu; Lemma on c-transform properties (ii))."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from scipy.interpolate import RegularGridInterpolator

from oracle import bfm as ob


def neumann_laplacian_apply(g):
    """Second-difference Laplacian with reflecting (zero-flux) ghost cells,
    applied directly, axis by axis."""
    out = np.zeros_like(g)
    for a, n in enumerate(g.shape):
        h2 = (1.0 / n) ** 2
        gp = np.concatenate([np.take(g, [0], axis=a), g, np.take(g, [n - 1], axis=a)], axis=a)
        lo = np.take(gp, np.arange(0, n), axis=a)
        hi = np.take(gp, np.arange(2, n + 2), axis=a)
        out += (lo - 2 * g + hi) / h2
    return out


def neumann_matrix(shape):
    mats = []
    for n in shape:
        main = -2.0 * np.ones(n)
        main[0] = main[-1] = -1.0
        L = sp.diags([np.ones(n - 1), main, np.ones(n - 1)], [-1, 0, 1]) * (n * n)
        mats.append(L.tocsr())
    A = None
    for a in range(len(shape)):
        term = None
        for b, n in enumerate(shape):
            m = mats[b] if a == b else sp.identity(n, format="csr")
            term = m if term is None else sp.kron(term, m, format="csr")
        A = term if A is None else A + term
    return A


@pytest.mark.parametrize("shape", [(16,), (24, 20), (12, 18), (6, 8, 10)])
def test_poisson_stencil_residual(shape):
    f = np.random.default_rng(1).normal(size=shape)
    g, G = ob.poisson_neumann(f)
    res = -neumann_laplacian_apply(g) - (f - f.mean())
    assert np.max(np.abs(res)) <= 1e-10 * np.max(np.abs(f))
    assert abs(g.mean()) <= 1e-13 * np.max(np.abs(g))


@pytest.mark.parametrize("shape", [(20, 14), (5, 6, 7)])
def test_poisson_sparse_direct(shape):
    f = np.random.default_rng(2).normal(size=shape)
    g, G = ob.poisson_neumann(f)
    A = neumann_matrix(shape)
    N = A.shape[0]
    # bordered system [ -A  1 ; 1^T 0 ] [g ; c] = [f - mean f ; 0]
    ones = sp.csr_matrix(np.ones((N, 1)))
    K = sp.bmat([[-A, ones], [ones.T, None]], format="csc")
    rhs = np.concatenate([(f - f.mean()).ravel(), [0.0]])
    sol = spla.spsolve(K, rhs)
    assert np.max(np.abs(sol[:N].reshape(shape) - g)) <= 1e-10 * np.max(np.abs(g))


@pytest.mark.parametrize("shape", [(32, 24), (6, 9, 8)])
def test_G_is_dirichlet_energy(shape):
    # G = vol * sum f g = vol * sum over edges |difference quotient of g|^2
    # (summation by parts with zero flux through the faces).
    f = np.random.default_rng(4).normal(size=shape)
    g, G = ob.poisson_neumann(f)
    vol = ob.cell_vol(shape)
    E = 0.0
    for a, n in enumerate(shape):
        E += np.sum((np.diff(g, axis=a) * n) ** 2)
    assert abs(G - vol * E) <= 1e-11 * abs(G)
    assert abs(G - vol * np.sum((f - f.mean()) * g)) <= 1e-11 * abs(G)


def _rand_map(shape, seed, amp=0.2):
    rng = np.random.default_rng(seed)
    xs = ob.centres(shape)
    T = []
    for a, n in enumerate(shape):
        h = 1.0 / n
        t = xs[a] + amp * rng.uniform(-1, 1, size=shape)
        T.append(np.clip(t, 0.5 * h, 1 - 0.5 * h))
    return T


@pytest.mark.parametrize("shape", [(32, 32), (16, 20), (8, 10, 12), (40,)])
def test_pushforward_mass_and_adjoint(shape):
    rng = np.random.default_rng(7)
    mu = rng.uniform(0, 2, size=shape)
    T = _rand_map(shape, 8)
    rho = ob.pushforward(mu, T)
    assert abs(rho.sum() - mu.sum()) <= 1e-13 * mu.sum()
    assert np.all(rho >= 0)
    # adjointness: sum_y rho(y) f(y) = sum_x mu(x) (I f)(T x), I = multilinear
    f = rng.normal(size=shape)
    axes = [(np.arange(n) + 0.5) / n for n in shape]
    interp = RegularGridInterpolator(axes, f, method="linear")
    pts = np.stack([t.ravel() for t in T], axis=1)
    lhs = np.sum(rho * f)
    rhs = np.sum(mu.ravel() * interp(pts))
    assert abs(lhs - rhs) <= 1e-12 * np.sum(np.abs(mu))


def test_pushforward_identity_and_shift():
    shape = (24, 20)
    rng = np.random.default_rng(9)
    mu = np.zeros(shape)
    mu[6:14, 5:12] = rng.uniform(0.5, 1.5, size=(8, 7))
    xs = ob.centres(shape)
    T = [xs[0] + np.zeros(shape), xs[1] + np.zeros(shape)]
    assert np.max(np.abs(ob.pushforward(mu, T) - mu)) <= 1e-15
    k = (3, -2)
    T = [xs[0] + k[0] / shape[0] + np.zeros(shape), xs[1] + k[1] / shape[1] + np.zeros(shape)]
    rho = ob.pushforward(mu, T)
    expect = np.roll(np.roll(mu, 3, axis=0), -2, axis=1)
    assert np.max(np.abs(rho - expect)) <= 1e-13


def test_map_of_linear_potential():
    # p^c(x) = -a.x gives T(x) = x + a exactly (central and one-sided
    # differences are exact on linear functions); clamped at the box.
    shape = (16, 12)
    xs = ob.centres(shape)
    a = (0.125, -1 / 6)
    pc = -(a[0] * xs[0] + a[1] * xs[1]) + np.zeros(shape)
    T = ob.transport_map(pc)
    for ax in range(2):
        h = 1.0 / shape[ax]
        expect = np.clip(xs[ax] + a[ax], 0.5 * h, 1 - 0.5 * h) + np.zeros(shape)
        assert np.max(np.abs(T[ax] - expect)) <= 1e-14
