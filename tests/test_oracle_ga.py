"""Pins for the oracle's plain H^1 gradient ascent: the scheme Section 4.3
compares the back-and-forth method with (Tables 5 and 6),
phi_{n+1/2} = phi_n + sigma grad J(phi_n), phi_{n+1} = (phi_{n+1/2})^cc.

The pins lean on facts that hold for the scheme whatever its step sizes:
every iterate after the first is c-concave, its c-transform is the inner
transform of the step that made it (f^ccc = f^c), the double transform never
lowers J, duals stay below the exact discrete optimum, and on the Section 4.3
examples the dual reaches the exact cost."""
import json
import os

import numpy as np
import pytest

from oracle import bfm as ob
from paper_1905_12154_amd import workloads as wl

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_examples.json")))


def _random_pair(shape, seed):
    rng = np.random.default_rng(seed)
    mu = rng.uniform(0.2, 2.0, size=shape)
    nu = rng.uniform(0.2, 2.0, size=shape)
    mu /= mu.sum() * ob.cell_vol(shape)
    nu /= nu.sum() * ob.cell_vol(shape)
    return mu, nu


@pytest.mark.parametrize("shape,iters", [((8, 6), 1), ((8, 6), 7), ((5, 4, 6), 4)])
def test_iterates_are_c_concave_and_psi_is_their_transform(shape, iters):
    # phi_{n+1} = (phi_{n+1/2})^cc is c-concave: (phi^c)^c = phi.  The returned
    # psi must be phi^c although the loop never transforms phi_{n+1} itself.
    # Checked with the non-separable brute-force transform of the definition.
    mu, nu = _random_pair(shape, 5)
    res = ob.solve_ga(mu, nu, ob.Params(max_iters=iters))
    assert res.iters == iters
    phic = ob.ctransform_bruteforce(res.phi)
    assert np.max(np.abs(phic - res.psi)) <= 1e-13
    assert np.max(np.abs(ob.ctransform_bruteforce(phic) - res.phi)) <= 1e-13


def test_double_transform_never_lowers_the_dual():
    # J((phi_{n+1/2})^cc) >= J(phi_{n+1/2}) (the c-transform half of the
    # monotone chain of Section 3.2), for every step, with any step size.
    mu, nu = wl.config_c1()
    res = ob.solve_ga(mu, nu, ob.Params(max_iters=25))
    tr = res.trace
    assert len(tr) == 26
    for k in range(len(tr) - 1):
        assert tr[k]["J_half"] <= tr[k + 1]["dual"] + 1e-14


def test_first_step_is_the_phi_half_step_of_algorithm_1():
    # Iteration 0 of both schemes is the same gradient step on J from phi_0 = 0.
    mu, nu = wl.config_c1()
    b = ob.solve(mu, nu, ob.Params(max_iters=1))
    g = ob.solve_ga(mu, nu, ob.Params(max_iters=1))
    assert g.trace[0]["dual"] == b.trace[0]["dual"]
    assert g.trace[0]["J_half"] == b.trace[0]["J_half"]
    # sigma after the first step: the phi-step update, before any psi-step
    expect = ob.update_sigma(b.trace[0]["sigma"], b.trace[0]["J_half"] - b.trace[0]["dual"],
                             b.trace[0]["G"], ob.Params())
    assert g.trace[1]["sigma"] == expect


@pytest.mark.parametrize("shape,seed", [((12,), 1), ((5, 5), 2), ((3, 3, 3), 4)])
def test_weak_duality_and_feasibility(shape, seed):
    from test_oracle_solve import _lp_cost
    mu, nu = _random_pair(shape, seed)
    lp, C = _lp_cost(mu, nu)
    res = ob.solve_ga(mu, nu, ob.Params(max_iters=40))
    for e in res.trace:
        assert e["dual"] <= lp + 1e-12
    phi, psi = res.phi.ravel(), res.psi.ravel()
    assert np.max(psi[:, None] + phi[None, :] - C) <= 1e-13
    assert res.dual >= 0.5 * lp


def test_two_discs_reaches_the_exact_cost():
    # Section 4.3: translation of a disc by (1/2, 1/2), cost 1/4.
    mu, nu = wl.two_discs(64)
    res = ob.solve_ga(mu, nu, ob.Params(max_iters=80))
    exact = GOLD["two_discs"]["cost"]
    err = [abs(e["dual"] - exact) for e in res.trace]
    assert err[-1] <= 1e-12
    assert all(e["dual"] <= exact + 1e-13 for e in res.trace)


@pytest.mark.parametrize("case,n", [("two_discs", 64), ("square_to_four", 64)])
def test_back_and_forth_needs_fewer_iterations(case, n):
    # Tables 5 and 6: to the same error in the transport cost the
    # back-and-forth iteration needs several times fewer iterations.
    mu, nu = getattr(wl, case)(n)
    exact = GOLD[case]["cost"]

    def first(tr, tol):
        return next((e["iter"] for e in tr if abs(e["dual"] - exact) < tol), None)

    b = ob.solve(mu, nu, ob.Params(max_iters=10))
    g = ob.solve_ga(mu, nu, ob.Params(max_iters=200))
    nb, ng = first(b.trace, 1e-4), first(g.trace, 1e-4)
    assert nb is not None and ng is not None
    assert ng >= 4 * nb
