"""Pins for the oracle's envelope gradient ``w2_gradients``: the first
variation of J (Lemma fact:derivative-J, Section 3) at a maximiser, i.e.
d W2^2 / d mu = 2 cell_volume (psi - mean psi) and
d W2^2 / d nu = 2 cell_volume (phi - mean phi), with W2^2 = 2 C(mu, nu) and
(phi, psi) the Kantorovich pair of Theorem thm:dual_problem (Section 2.1).

Three independent routes fix it:

* the exact discrete optimal transport (a linear programme solved by HiGHS):
  its value is piecewise linear in the marginals and, where the optimal basis
  does not change, its central differences along zero-mass directions equal
  the inner product with the LP's dual variables exactly -- so the formula,
  applied to the LP's maximiser, must reproduce them (the factor 2, the cell
  volume and which potential belongs to which density are all fixed here);
* closed forms of the continuous problem: a whole-cell translation by a has
  psi(x) = -a.x and phi(y) = a.y + const on the supports; N(m1, s1^2 I) to
  N(m2, s2^2 I) has psi(x) = (1 - r)|x|^2/2 + (r m1 - m2).x and
  phi(y) = (1 - 1/r)|y|^2/2 + (m2/r - m1).y, r = s2/s1 (T = x - grad psi);
* central differences of the oracle's own converged W2^2.  The back-and-forth
  fixed point with the finite-difference map and cloud-in-cell deposition is
  not the exact maximiser of the grid dual, so these agree only up to the
  discretisation; the test records that the disagreement shrinks as the grid
  is refined (about 3-5x per halving of h).
"""
import numpy as np
import pytest
from scipy.optimize import linprog

from oracle import bfm as ob
from paper_1905_12154_amd import workloads as wl


def _lp(mu, nu):
    """Exact discrete OT between the grid measures cell_volume*mu and
    cell_volume*nu for c = |x - y|^2 / 2: value and dual variables (psi on
    the mu side, phi on the nu side; d value / d mass = dual)."""
    shape = mu.shape
    C = ob.cost_matrix(shape)
    v = ob.cell_vol(shape)
    a, b = v * mu.ravel(), v * nu.ravel()
    N = a.size
    A_eq = np.zeros((2 * N, N * N))
    for i in range(N):
        A_eq[i, i * N:(i + 1) * N] = 1.0
        A_eq[N + i, i::N] = 1.0
    r = linprog(C.ravel(), A_eq=A_eq, b_eq=np.concatenate([a, b]), bounds=(0, None), method="highs")
    assert r.status == 0
    m = r.eqlin.marginals
    return r.fun, m[:N].reshape(shape), m[N:].reshape(shape)


def _result(phi, psi):
    z = np.zeros_like(phi)
    return ob.Result(phi=phi, psi=psi, T=[z] * phi.ndim, dual=0.0, primal=0.0, gap=0.0, G=0.0, sigma=0.0,
                     iters=0, converged=True)


def _zero_mass_direction(rho, rng):
    w = rng.normal(size=rho.shape)
    return rho * (w - (rho * w).sum() / rho.sum())


# The formula with plausible mistakes; each must fail the LP pin.
def _swapped(res, shape):
    v = ob.cell_vol(shape)
    return 2 * v * (res.phi - res.phi.mean()), 2 * v * (res.psi - res.psi.mean())


def _no_two(res, shape):
    g, h = ob.w2_gradients(res, shape)
    return 0.5 * g, 0.5 * h


def _no_volume(res, shape):
    g, h = ob.w2_gradients(res, shape)
    return g / ob.cell_vol(shape), h / ob.cell_vol(shape)


def _wrong_sign(res, shape):
    g, h = ob.w2_gradients(res, shape)
    return -g, -h


def _lp_pin_errors(grad_fn, shape, seed):
    rng = np.random.default_rng(seed)
    mu = rng.uniform(0.3, 2.0, size=shape)
    nu = rng.uniform(0.3, 2.0, size=shape)
    mu /= mu.sum() * ob.cell_vol(shape)
    nu /= nu.sum() * ob.cell_vol(shape)
    val, psi, phi = _lp(mu, nu)
    gmu, gnu = grad_fn(_result(phi, psi), shape)
    errs = []
    for which in (0, 1):
        for _ in range(3):
            v = _zero_mass_direction(mu if which == 0 else nu, rng)
            eps = 1e-6 / np.max(np.abs(v))
            if which == 0:
                fd = (_lp(mu + eps * v, nu)[0] - _lp(mu - eps * v, nu)[0]) / (2 * eps)
            else:
                fd = (_lp(mu, nu + eps * v)[0] - _lp(mu, nu - eps * v)[0]) / (2 * eps)
            an = float(((gmu if which == 0 else gnu) * v).sum())
            errs.append(abs(2.0 * fd - an) / abs(2.0 * fd))
    return errs


@pytest.mark.parametrize("shape,seed", [((4, 4), 1), ((3, 5), 2), ((9,), 3), ((2, 3, 2), 4)])
def test_lp_value_derivative_equals_formula_on_lp_potentials(shape, seed):
    errs = _lp_pin_errors(ob.w2_gradients, shape, seed)
    assert max(errs) <= 1e-5, errs


@pytest.mark.parametrize("wrong", [_swapped, _no_two, _no_volume, _wrong_sign])
def test_lp_pin_rejects_planted_mistakes(wrong):
    assert max(_lp_pin_errors(wrong, (4, 4), 1)) > 1e-2


def test_gradients_are_zero_mass():
    rng = np.random.default_rng(0)
    phi, psi = rng.normal(size=(6, 5)), rng.normal(size=(6, 5))
    gmu, gnu = ob.w2_gradients(_result(phi, psi), (6, 5))
    assert abs(gmu.sum()) <= 1e-15 and abs(gnu.sum()) <= 1e-15


def _interior(mask):
    out = mask.copy()
    for a in range(mask.ndim):
        out &= np.roll(mask, 1, axis=a) & np.roll(mask, -1, axis=a)
    return out


def _centred(f, sup):
    return f[sup] - f[sup].mean()


@pytest.mark.parametrize("shape,shift", [((48, 48), (7, -5)), ((40, 56), (-6, 9))])
def test_translation_closed_form(shape, shift):
    # mu(x) = nu(x + a), a = whole cells: psi = -a.x on supp mu, phi = a.y on
    # supp nu.  One ball: on a support with several components each component
    # may carry its own additive constant.
    mu, nu = wl.translated_pair(shape, shift, np.random.default_rng(11), k=1, rmin=0.12, rmax=0.16)
    res = ob.solve(mu, nu, ob.Params(max_iters=12))
    gmu, gnu = ob.w2_gradients(res, shape)
    v = ob.cell_vol(shape)
    xs = ob.centres(shape)
    a = [s / n for s, n in zip(shift, shape)]
    lin = sum(ai * x for ai, x in zip(a, xs)) + np.zeros(shape)
    for g, sup, exact in ((gmu, _interior(mu > 0), -lin), (gnu, _interior(nu > 0), lin)):
        err = np.max(np.abs(_centred(g, sup) - 2 * v * _centred(exact, sup)))
        scale = np.max(np.abs(2 * v * _centred(exact, sup)))
        # the discrete dual optimum is a polytope: potentials wobble by ~1e-3
        # of their range on the support (a swapped pair is off by 2x the range)
        assert err <= 1e-2 * scale, (err, scale)


def test_gaussian_closed_form():
    n = 128
    m1, s1 = np.array([0.42, 0.45]), 0.05
    m2, s2 = np.array([0.56, 0.52]), 0.06
    r = s2 / s1
    mu = wl.gaussian_mixture((n, n), [m1], [s1])
    nu = wl.gaussian_mixture((n, n), [m2], [s2])
    res = ob.solve(mu, nu, ob.Params(max_iters=40))
    gmu, gnu = ob.w2_gradients(res, (n, n))
    v = ob.cell_vol((n, n))
    xs = ob.centres((n, n))
    r2 = xs[0] ** 2 + xs[1] ** 2
    psi = 0.5 * (1 - r) * r2 + (r * m1[0] - m2[0]) * xs[0] + (r * m1[1] - m2[1]) * xs[1]
    phi = 0.5 * (1 - 1 / r) * r2 + (m2[0] / r - m1[0]) * xs[0] + (m2[1] / r - m1[1]) * xs[1]
    for g, rho, exact in ((gmu, mu, psi), (gnu, nu, phi)):
        sup = rho > 0.2 * rho.max()
        ref = 2 * v * _centred(exact, sup)
        err = np.max(np.abs(_centred(g, sup) - ref))
        # grid error ~1e-3 of the potential's range; a swapped pair or a wrong
        # factor is off by O(1) of it
        assert err <= 1e-2 * np.max(np.abs(ref)), (err, np.max(np.abs(ref)))


def _fd_errors(n, seed):
    """Relative disagreement of central differences of the converged W2^2
    with the envelope gradient, three zero-mass smooth directions per
    density (multiplicative, max |eps v / rho| = 2e-2).  The perturbed solves
    start from the base solution so that all three runs sit on the same
    stretch of the slow final approach (the gradient of the grid dual does not
    vanish at the fixed point of the discrete iteration, and W2^2 keeps
    creeping up by ~1e-7 per iteration)."""
    mu = wl.gaussian_mixture((n, n), [(0.4, 0.45)], [0.08])
    nu = wl.gaussian_mixture((n, n), [(0.55, 0.5)], [0.06])
    base = ob.solve(mu, nu, ob.Params(max_iters=1000))
    gmu, gnu = ob.w2_gradients(base, mu.shape)
    prm = ob.Params(max_iters=200, sigma0=base.sigma)
    rng = np.random.default_rng(seed)
    xs = ob.centres(mu.shape)
    out = {"mu": [], "nu": []}
    for which, rho, g in (("mu", mu, gmu), ("nu", nu, gnu)):
        for _ in range(3):
            k = rng.integers(1, 4, size=2)
            ph = rng.uniform(0, 2 * np.pi, size=2)
            w = np.cos(np.pi * k[0] * xs[0] + ph[0]) * np.cos(np.pi * k[1] * xs[1] + ph[1])
            v = rho * (w - (rho * w).sum() / rho.sum())
            eps = 2e-2 / np.max(np.abs(v) / rho)
            if which == "mu":
                wp = ob.solve(mu + eps * v, nu, prm, phi_init=base.phi).w2sq
                wm = ob.solve(mu - eps * v, nu, prm, phi_init=base.phi).w2sq
            else:
                wp = ob.solve(mu, nu + eps * v, prm, phi_init=base.phi).w2sq
                wm = ob.solve(mu, nu - eps * v, prm, phi_init=base.phi).w2sq
            fd = (wp - wm) / (2 * eps)
            out[which].append(abs(fd - float((g * v).sum())) / abs(fd))
    return {k: float(np.mean(e)) for k, e in out.items()}


def test_central_differences_converge_with_the_grid():
    e = {n: _fd_errors(n, 0) for n in (16, 32, 64)}
    print("mean relative FD disagreement", e)
    # measured: mu 0.093 / 0.014 / 0.0029, nu 0.139 / 0.072 / 0.011 at 16 / 32 / 64:
    # at least first order in h over the two halvings
    for which in ("mu", "nu"):
        assert e[32][which] <= 0.75 * e[16][which]
        assert e[64][which] <= 0.5 * e[32][which]
        assert e[64][which] <= 0.25 * e[16][which]
    assert e[64]["mu"] <= 1e-2 and e[64]["nu"] <= 3e-2
