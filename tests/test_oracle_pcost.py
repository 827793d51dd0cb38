"""Pins for the oracle's separable power costs c(x, y) = sum_a |x_a - y_a|^{p_a} / p_a
(eq. p_costs; Section 4.1 for the separable c-transform of such costs,
Section 4.3 for the experiment with two pairs of discs).

The pins: the separable transform against the non-separable definition, the
c-transform identities, the map of a linear potential (a translation whose
length inverts h'), the exact cost of translations (Jensen: for a convex
translation-invariant cost, translating is optimal), weak duality against the
exact discrete LP, and the paper's statement that with p = 1.1 on one axis and
p = 3 on the other the discs move along one axis only."""
import numpy as np
import pytest
from scipy.optimize import linprog

from oracle import bfm as ob
from paper_1905_12154_amd import workloads as wl


@pytest.mark.parametrize("shape,powers", [((9,), (1.3,)), ((6, 5), (1.5, 3.0)), ((7, 4), (1.1, 2.0)),
                                          ((4, 3, 5), (1.5, 3.0, 1.2)), ((5, 4, 3), (2.0, 2.5, 4.0))])
def test_separable_transform_equals_definition(shape, powers):
    rng = np.random.default_rng(len(shape) * 10 + 1)
    for scale in (0.05, 1.0):
        f = scale * rng.normal(size=shape)
        a = ob.ctransform(f, powers)
        b = ob.ctransform_bruteforce(f, powers)
        assert np.max(np.abs(a - b)) <= 1e-14


def test_power_two_is_the_quadratic_cost():
    rng = np.random.default_rng(2)
    u = rng.normal(size=(7, 33))
    assert np.max(np.abs(ob.line_min_p(u, 1, 2.0) - ob.line_min(u, 1))) <= 1e-15
    assert np.max(np.abs(ob.line_min_p(u, 0, 2.0) - ob.line_min(u, 0))) <= 1e-15


@pytest.mark.parametrize("powers", [(1.5, 3.0), (1.1, 1.7)])
def test_c_transform_identities(powers):
    # Lemma on c-transform properties: f <= f^cc and f^ccc = f^c, any cost
    rng = np.random.default_rng(3)
    f = rng.normal(scale=0.3, size=(24, 20))
    fc = ob.ctransform(f, powers)
    fcc = ob.ctransform(fc, powers)
    assert np.all(f <= fcc + 1e-14)
    assert np.max(np.abs(ob.ctransform(fcc, powers) - fc)) <= 1e-14


def test_map_of_a_linear_potential_is_a_translation():
    # phi(y) = s . y with s_a = h_a'(k_a / n_a): the minimiser of
    # h(y - x) - phi(y) is y = x + k / n wherever that point is on the grid,
    # so T(x) = x - (grad h)^{-1}(grad phi^c(x)) = x + k / n there.
    shape, powers, k = (40, 36), (1.5, 3.0), (3, -2)
    xs = ob.centres(shape)
    s = [np.sign(kk) * abs(kk / n) ** (p - 1.0) for kk, n, p in zip(k, shape, powers)]
    phi = s[0] * xs[0] + s[1] * xs[1]
    T = ob.transport_map(ob.ctransform(phi, powers), powers)
    i0 = np.arange(shape[0])[:, None]
    i1 = np.arange(shape[1])[None, :]
    # cells whose stencil neighbours all have their minimiser on the grid
    ok = ((i0 + k[0] - 1 >= 0) & (i0 + k[0] + 1 < shape[0]) & (i0 >= 1) & (i0 <= shape[0] - 2)
          & (i1 + k[1] - 1 >= 0) & (i1 + k[1] + 1 < shape[1]) & (i1 >= 1) & (i1 <= shape[1] - 2))
    assert ok.sum() > 500
    for a in range(2):
        assert np.max(np.abs((T[a] - xs[a] - k[a] / shape[a])[ok])) <= 1e-12


def test_primal_cost_of_a_translation():
    shape, powers = (16, 12), (1.5, 2.5)
    mu = wl.normalise(np.ones(shape))
    xs = ob.centres(shape)
    a = (0.1, -0.2)
    P = ob.primal_cost(mu, [xs[0] + a[0], xs[1] + a[1]], powers)
    assert abs(P - (0.1 ** 1.5 / 1.5 + 0.2 ** 2.5 / 2.5)) <= 1e-15


@pytest.mark.parametrize("shape,shift,powers,iters", [((48, 48), (7, -5), (1.5, 3.0), 40),
                                                      ((40, 56), (-6, 9), (3.0, 1.25), 60),
                                                      ((24, 24, 24), (3, -2, 4), (1.5, 2.0, 3.0), 80)])
def test_translation_exact_cost(shape, shift, powers, iters):
    # mu(x) = nu(x + a): for any coupling, Jensen gives sum pi h(y - x) >=
    # h(mean displacement) = h(a), which the translation attains.
    radii = (0.06, 0.1) if len(shape) == 2 else (0.15, 0.2)
    mu, nu = wl.translated_pair(shape, shift, np.random.default_rng(11), rmin=radii[0], rmax=radii[1])
    res = ob.solve(mu, nu, ob.Params(max_iters=iters, powers=powers))
    exact = sum(abs(s / n) ** p / p for s, n, p in zip(shift, shape, powers))
    assert min(abs(e["dual"] - exact) for e in res.trace) <= 1e-12
    assert all(e["dual"] <= exact + 1e-13 for e in res.trace)


@pytest.mark.parametrize("shape,powers,seed", [((12,), (1.5,), 1), ((5, 5), (1.5, 3.0), 2),
                                               ((3, 3, 3), (1.2, 2.0, 2.5), 4)])
def test_weak_duality_against_lp(shape, powers, seed):
    rng = np.random.default_rng(seed)
    mu = rng.uniform(0.2, 2.0, size=shape)
    nu = rng.uniform(0.2, 2.0, size=shape)
    mu /= mu.sum() * ob.cell_vol(shape)
    nu /= nu.sum() * ob.cell_vol(shape)
    pts = np.stack([x.ravel() for x in np.meshgrid(*[(np.arange(n) + 0.5) / n for n in shape],
                                                     indexing="ij")], axis=1)
    C = np.zeros((pts.shape[0], pts.shape[0]))
    for a, p in enumerate(powers):
        C += np.abs(pts[:, None, a] - pts[None, :, a]) ** p / p
    a_, b_ = mu.ravel() / mu.sum(), nu.ravel() / nu.sum()
    N = a_.size
    A = np.zeros((2 * N, N * N))
    for i in range(N):
        A[i, i * N:(i + 1) * N] = 1.0
        A[N + i, i::N] = 1.0
    lp = linprog(C.ravel(), A_eq=A, b_eq=np.concatenate([a_, b_]), bounds=(0, None), method="highs")
    assert lp.status == 0
    res = ob.solve(mu, nu, ob.Params(max_iters=30, powers=powers))
    for e in res.trace:
        assert e["dual"] <= lp.fun + 1e-12
    phi, psi = res.phi.ravel(), res.psi.ravel()
    assert np.max(psi[:, None] + phi[None, :] - C) <= 1e-13
    assert res.dual >= 0.5 * lp.fun


def test_crossing_discs_move_along_the_cheap_axis_only():
    # Section 4.3 (general costs): with exponent 3 on one axis and 1.1 on the
    # other, moving 1/2 along the first costs (1/2)^3/3 = 1/24 and along the
    # second (1/2)^1.1/1.1 = 0.42, so the discs translate along the first
    # axis only, at cost 1/24; with equal exponents mass moves along both.
    mu, nu = wl.crossing_discs(64)
    xs = ob.centres(mu.shape)
    sup = mu > 0
    res = ob.solve(mu, nu, ob.Params(max_iters=40, powers=(3.0, 1.1)))
    assert min(abs(e["dual"] - 1.0 / 24.0) for e in res.trace) <= 1e-12
    assert np.max(np.abs(res.T[1] - xs[1])[sup]) <= 0.25 / 64
    assert np.mean(np.abs(res.T[0] - xs[0])[sup]) >= 0.49
    q = ob.solve(mu, nu, ob.Params(max_iters=40))
    assert np.mean(np.abs(q.T[1] - xs[1])[sup]) >= 0.15
    assert q.dual < 0.125   # cheaper than translating each disc by 1/2
