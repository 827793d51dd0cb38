"""Pins for the oracle's step rule (Section 4.2) and whole back-and-forth loop
(Algorithm 1) against values the paper prints (Section 4.3) and facts the
mathematics fixes (weak duality, c-transform monotonicity, closed forms)."""
import json
import os

import numpy as np
import pytest
from scipy.optimize import linprog

from oracle import bfm as ob
from paper_1905_12154_amd import workloads as wl

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_examples.json")))


# ---------------------------------------------------------------- step rule

def test_step_rule_constants_match_paper():
    p = ob.Params()
    g = GOLD["step_rule"]
    assert (p.beta1, p.beta2, p.alpha1, p.alpha2, p.sigma_min) == (
        g["beta1"], g["beta2"], g["alpha1"], g["alpha2"], g["sigma_min"])
    mu = np.ones((4, 4)) * 2.0
    nu = np.ones((4, 4)) * 0.5
    assert ob.initial_sigma(mu, nu) == g["sigma0_factor"] * min(1 / 2.0, 1 / 0.5)


@pytest.mark.parametrize("sigma,inc,G,expect", [
    (1.0, 0.10, 1.0, 0.8),      # increase below beta1*sigma*G: shrink by alpha2
    (1.0, 0.25, 1.0, 1.0),      # exactly beta1*sigma*G: inside the band, keep
    (1.0, 0.50, 1.0, 1.0),      # inside the band
    (1.0, 0.75, 1.0, 1.0),      # exactly beta2*sigma*G: keep
    (1.0, 0.90, 1.0, 1.25),     # above beta2*sigma*G: grow by alpha1
    (2.0, 0.30, 1.0, 1.6),      # band scales with sigma: [0.5, 1.5]; 0.3 below it -> shrink
    (0.011, -1.0, 1.0, 0.01),   # shrink floored at sigma_min
    (0.005, -1.0, 1.0, 0.01),   # below the floor already: the floor applies
])
def test_step_rule_scripted(sigma, inc, G, expect):
    p = ob.Params()
    got = ob.update_sigma(sigma, inc, G, p)
    assert got == pytest.approx(expect, rel=0, abs=1e-15)


def test_step_rule_sequence():
    # A scripted trajectory: hand-computed from the Section 4.2 rule.
    p = ob.Params()
    s = 1.0
    seq = [(0.1, 1.0), (0.1, 1.0), (2.0, 1.0), (0.5, 1.0), (0.0, 0.0)]
    out = []
    for inc, G in seq:
        s = ob.update_sigma(s, inc, G, p)
        out.append(s)
    # 1 -> 0.8 -> 0.64 (0.1 < 0.16) -> 0.8 (2 > 0.48) -> 0.8 (0.5 in [0.2,0.6]) -> 0.8 (0 in [0,0])
    assert out == pytest.approx([0.8, 0.64, 0.8, 0.8, 0.8], abs=1e-15)


# ------------------------------------------------------- paper's examples

def _interior(mask):
    out = mask.copy()
    for a in range(mask.ndim):
        out &= np.roll(mask, 1, axis=a) & np.roll(mask, -1, axis=a)
    return out


def _errors(res, exact):
    return [abs(e["dual"] - exact) for e in res.trace]


def test_two_discs_exact_cost():
    mu, nu = wl.two_discs(64)
    res = ob.solve(mu, nu, ob.Params(max_iters=8))
    err = _errors(res, GOLD["two_discs"]["cost"])
    assert min(err) <= 1e-12
    assert err[-1] <= 1e-12
    # the map is the translation by (1/2, 1/2) on the support of mu (cells
    # whose stencil neighbours are in the support too)
    sup = _interior(mu > 0)
    xs = ob.centres(mu.shape)
    # Discrete optimal potentials are not unique, so the finite-difference
    # map may wobble within a fraction of a cell on the support.
    for a in range(2):
        assert np.max(np.abs((res.T[a] - xs[a])[sup] - 0.5)) <= 0.25 / mu.shape[a]


def test_square_to_four_exact_cost():
    mu, nu = wl.square_to_four(64)
    res = ob.solve(mu, nu, ob.Params(max_iters=10))
    err = _errors(res, GOLD["square_to_four"]["cost"])
    assert err[-1] <= 1e-12
    # the dual value is a lower bound of the discrete optimum at every step
    assert all(e["dual"] <= GOLD["square_to_four"]["cost"] + 1e-13 for e in res.trace)


def test_two_balls_exact_cost():
    mu, nu = wl.two_balls(32)
    res = ob.solve(mu, nu, ob.Params(max_iters=10))
    assert _errors(res, GOLD["two_balls"]["cost"])[-1] <= 1e-12


def test_cube_to_eight_exact_cost():
    mu, nu = wl.cube_to_eight(32)
    res = ob.solve(mu, nu, ob.Params(max_iters=10))
    assert _errors(res, GOLD["cube_to_eight"]["cost"])[-1] <= 1e-12


@pytest.mark.parametrize("shape,shift,radii", [((48, 48), (7, -5), (0.06, 0.1)),
                                               ((40, 56), (-6, 9), (0.06, 0.1)),
                                               ((24, 24, 24), (3, -2, 4), (0.15, 0.2))])
def test_random_translation(shape, shift, radii):
    # Section 4.3: mu(x) = nu(x + a) -> T = x + a, cost |a|^2 / 2 (a = whole cells)
    mu, nu = wl.translated_pair(shape, shift, np.random.default_rng(11), rmin=radii[0], rmax=radii[1])
    res = ob.solve(mu, nu, ob.Params(max_iters=12))
    a2 = sum((s / n) ** 2 for s, n in zip(shift, shape))
    assert min(abs(e["dual"] - 0.5 * a2) for e in res.trace) <= 1e-12
    assert all(e["dual"] <= 0.5 * a2 + 1e-13 for e in res.trace)
    if len(shape) == 3:
        return
    assert abs(res.dual - 0.5 * a2) <= 1e-12
    sup = _interior(mu > 0)
    xs = ob.centres(shape)
    for a, (s, n) in enumerate(zip(shift, shape)):
        assert np.max(np.abs((res.T[a] - xs[a])[sup] - s / n)) <= 0.25 / n


# ----------------------------------------------------------- weak duality

def _lp_cost(mu, nu):
    """Exact discrete optimal transport between grid measures (HiGHS)."""
    shape = mu.shape
    xs = np.stack([x.ravel() for x in np.meshgrid(*[(np.arange(n) + 0.5) / n for n in shape],
                                                    indexing="ij")], axis=1)
    C = 0.5 * ((xs[:, None, :] - xs[None, :, :]) ** 2).sum(-1)
    a = mu.ravel() / mu.sum()
    b = nu.ravel() / nu.sum()
    N = a.size
    A_eq = np.zeros((2 * N, N * N))
    for i in range(N):
        A_eq[i, i * N:(i + 1) * N] = 1.0
        A_eq[N + i, i::N] = 1.0
    r = linprog(C.ravel(), A_eq=A_eq, b_eq=np.concatenate([a, b]), bounds=(0, None), method="highs")
    assert r.status == 0
    return r.fun, C


@pytest.mark.parametrize("shape,seed", [((12,), 1), ((5, 5), 2), ((6, 4), 3), ((3, 3, 3), 4)])
def test_weak_duality_against_lp(shape, seed):
    rng = np.random.default_rng(seed)
    mu = rng.uniform(0.2, 2.0, size=shape)
    nu = rng.uniform(0.2, 2.0, size=shape)
    mu /= mu.sum() * ob.cell_vol(shape)
    nu /= nu.sum() * ob.cell_vol(shape)
    lp, C = _lp_cost(mu, nu)
    res = ob.solve(mu, nu, ob.Params(max_iters=25))
    for e in res.trace:
        assert e["dual"] <= lp + 1e-12
    # the returned pair is feasible: phi(y) + psi(x) <= c(x, y) for all pairs
    phi, psi = res.phi.ravel(), res.psi.ravel()
    assert np.max(psi[:, None] + phi[None, :] - C) <= 1e-13
    # the ascent makes real progress from D_0 = 0 (the remaining distance to
    # the LP value is the discretisation of the pushforward on a tiny grid)
    assert res.dual >= 0.5 * lp


def test_monotone_c_transform_half_of_chain():
    # Section 3.2: J(phi_{n+1/2}) <= I(psi_{n+1/2}) and I(psi_{n+1}) <= J(phi_{n+1})
    # hold for every iterate (the c-transform steps never decrease D).
    mu, nu = wl.config_c1()
    res = ob.solve(mu, nu, ob.Params(max_iters=20))
    tr = res.trace
    for k in range(len(tr) - 1):
        assert tr[k]["J_half"] <= tr[k]["I_old"] + 1e-14
        assert tr[k]["I_new"] <= tr[k + 1]["dual"] + 1e-14


def test_c1_dual_nondecreasing_and_converges():
    # Empirical on the smooth C1 mixture (the full chain of the ascent
    # proposition needs Hessian bounds the iterates need not satisfy).  At 64^2
    # the primal-dual discrepancy of the finite-difference map has an O(h^2)
    # floor, so the gap settles near 1e-4 while D keeps creeping up.
    mu, nu = wl.config_c1()
    res = ob.solve(mu, nu, ob.Params(max_iters=60))
    d = [e["dual"] for e in res.trace]
    assert all(d[k + 1] >= d[k] - 1e-12 for k in range(len(d) - 1))
    assert res.trace[-1]["G"] <= 1e-3 * res.trace[0]["G"]
    assert res.gap <= 2e-4


# ------------------------------------------------------ Gaussian and 1D

def test_gaussian_to_gaussian_affine_map():
    # N(m1, s1^2 I) -> N(m2, s2^2 I): T = m2 + (s2/s1)(x - m1),
    # cost (|m1 - m2|^2 + d (s1 - s2)^2) / 2.
    n = 128
    m1, s1 = np.array([0.42, 0.45]), 0.04
    m2, s2 = np.array([0.56, 0.52]), 0.05
    mu = wl.gaussian_mixture((n, n), [m1], [s1])
    nu = wl.gaussian_mixture((n, n), [m2], [s2])
    res = ob.solve(mu, nu, ob.Params(max_iters=40))
    exact = 0.5 * (np.sum((m1 - m2) ** 2) + 2 * (s1 - s2) ** 2)
    # discretisation-level agreement: a dropped term or a wrong sign in the
    # loop moves D by ~1e-2 here, the grid error is ~1e-4
    assert abs(res.dual - exact) <= 2e-4
    xs = ob.centres((n, n))
    sup = mu > 0.3 * mu.max()
    for a in range(2):
        Ta = m2[a] + (s2 / s1) * (xs[a] - m1[a]) + np.zeros((n, n))
        assert np.max(np.abs(res.T[a] - Ta)[sup]) <= 1.0 / n


def test_one_dimensional_quantile_coupling():
    # 1D: the monotone (north-west corner) coupling of the grid measures is
    # the exact discrete optimum; the dual stays below it and approaches it.
    n = 96
    x = (np.arange(n) + 0.5) / n
    mu = np.exp(-(x - 0.35) ** 2 / (2 * 0.06 ** 2)) + 0.05
    nu = np.exp(-(x - 0.6) ** 2 / (2 * 0.09 ** 2)) + 0.05
    mu /= mu.sum() / n
    nu /= nu.sum() / n
    a, b = mu / n, nu / n
    i = j = 0
    ra, rb = a[0], b[0]
    cost = 0.0
    while i < n and j < n:
        m = min(ra, rb)
        cost += m * 0.5 * (x[i] - x[j]) ** 2
        ra -= m
        rb -= m
        if ra <= 1e-18:
            i += 1
            ra = a[i] if i < n else 0
        if rb <= 1e-18:
            j += 1
            rb = b[j] if j < n else 0
    res = ob.solve(mu, nu, ob.Params(max_iters=40))
    assert all(e["dual"] <= cost + 1e-13 for e in res.trace)
    assert cost - res.dual <= 1e-4
