"""The solver's production kernels against the float64 oracle, and the error
paths of the controller.

* Algorithm 1 with the Section 4.2 step rule, run in float64 with the launch
  shapes the float32 production path uses: persistent c-transform workgroups,
  the column-blocked two-pass 2D transform and the sums fused into the passes
  that write p and q.  (Untuned float64 plans pick the one-group-per-workgroup
  kernel, so the ordinary parity tests do not reach these kernels.)
* Displacement interpolation (Section 4.3) in float32, element by element.
* A non-finite value in the device state (BFM_ENUMERIC).
* The count of step-size updates that held sigma at sigma_min, pinned to the
  oracle's own step rule.
"""
import numpy as np
import pytest
import torch

from oracle import bfm as ob
from paper_1905_12154_amd import bfm, workloads as wl

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def cuda(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def host(t):
    return t.detach().double().cpu().numpy()


@pytest.mark.parametrize("shape,C", [((64, 64), 4), ((256, 256), 16), ((512, 512), 16), ((192, 256), 16)])
def test_solve_parity_production_shapes_f64(shape, C):
    rng = np.random.default_rng(21)
    mu = wl.random_gaussian_mixture(shape, 3, rng)
    nu = wl.random_gaussian_mixture(shape, 4, rng)
    plan = bfm.Plan(shape, torch.float64, max_iters=12)
    plan.set_tuning([(C, 4, 2), (C, 0, 2)])
    assert plan.tuning() == [(C, 4, 2), (C, 0, 2)]
    # the column-blocked two-pass transform applies to this plan (it raises
    # BFM_EUNSUPPORTED where the persistent blocked kernels do not apply)
    tmu, tnu = cuda(mu), cuda(nu)
    blk = plan.ctransform_pass(tmu, 0)
    full = plan.ctransform_pass(blk, 1)
    assert float((full - plan.ctransform(tmu)).abs().max()) <= 1e-13 * float(full.abs().max())
    r = plan.solve(tmu, tnu)
    o = ob.solve(mu, nu, ob.Params(max_iters=12))
    assert r.iters == o.iters == 12
    assert abs(r.dual - o.dual) <= 1e-10
    assert abs(r.w2sq - o.w2sq) <= 1e-5 * abs(o.w2sq)
    assert abs(r.primal - o.primal) <= 1e-10
    assert abs(r.gap - o.gap) <= 1e-10 + 1e-8 * o.gap
    assert r.sigma == pytest.approx(o.sigma, rel=1e-12)
    for a in range(2):
        assert np.max(np.abs(host(r.T[a]) - o.T[a])) * shape[a] <= 1e-3
    # full-support densities: potentials are unique up to the removed mean
    assert np.max(np.abs(host(r.phi) - o.phi)) <= 1e-7
    assert np.max(np.abs(host(r.psi) - o.psi)) <= 1e-7



def test_solve_parity_production_shapes_3d_f64():
    """3D with persistent prefetching workgroups on every axis (the launch
    shapes of the float32 384^3 path), in float64 against the oracle,
    including the per-iteration trace of J(phi_{n+1/2}) and I(psi_{n+1})."""
    rng = np.random.default_rng(22)
    shape = (48, 36, 32)
    mu = wl.random_gaussian_mixture(shape, 3, rng)
    nu = wl.random_gaussian_mixture(shape, 4, rng)
    plan = bfm.Plan(shape, torch.float64, max_iters=8)
    plan.set_tuning([(4, 4, 2), (4, 4, 2), (4, 0, 2)])
    r = plan.solve(cuda(mu), cuda(nu))
    o = ob.solve(mu, nu, ob.Params(max_iters=8))
    assert r.iters == o.iters == 8
    assert abs(r.dual - o.dual) <= 1e-10
    assert abs(r.primal - o.primal) <= 1e-10
    assert r.sigma == pytest.approx(o.sigma, rel=1e-12)
    for a in range(3):
        assert np.max(np.abs(host(r.T[a]) - o.T[a])) * shape[a] <= 1e-3
    tr = plan.trace(DEV)
    ot = o.trace
    for k in range(8):
        assert tr[k]["J_half"] == pytest.approx(ot[k]["J_half"], rel=1e-10, abs=1e-12)
        assert tr[k]["I_new"] == pytest.approx(ot[k]["I_new"], rel=1e-10, abs=1e-12)

def test_interpolant_f32_elementwise():
    """float32 frames against the float64 oracle on the same float32 input
    potential, element by element.  The float32 c-transform is exact to a few
    ulps of the potential's scale (here ~0.2, so ~5e-8); the map's central
    difference multiplies that by n / 2, so T moves by up to ~5e-8 n^2 / 2
    cells (~2e-3 cells at 256^2), which shifts each multilinear weight by as
    much and each frame value by a few times that fraction of the largest
    deposited mass.  Bar: 1e-2 of the frame's maximum."""
    mu, _ = wl.config_c5_pair(1, 256)
    mu32 = mu.astype(np.float32)
    xs = ob.centres(mu.shape)
    phi = (0.12 * xs[0] ** 2 + 0.1 * xs[1] ** 2 - 0.05 * xs[0] * xs[1]
           + 0.01 * np.sin(6 * xs[0]) * np.cos(5 * xs[1])).astype(np.float32)
    times = [0.0, 0.25, 0.5, 0.75, 1.0]
    got = host(bfm.interpolate(cuda(phi, torch.float32), cuda(mu32, torch.float32), times))
    pco = ob.ctransform(phi.astype(np.float64))
    worst = 0.0
    for k, t in enumerate(times):
        ref = ob.displacement_interpolant(mu32.astype(np.float64), pco, t)
        err = np.max(np.abs(got[k] - ref)) / np.max(ref)
        worst = max(worst, err)
        assert err <= 1e-2, (t, err)
    print("float32 frame error / max", worst)
    # t = 0 deposits every cell onto itself: exact up to float32 rounding of mu
    assert np.max(np.abs(got[0] - mu32)) <= 1e-6 * np.max(mu32)


def test_nonfinite_state_is_reported():
    """A NaN in the warm start reaches J(phi_0) at the first head; the
    controller sets its non-finite flag, stops the loop and the solve returns
    BFM_ENUMERIC (validation accepts phi_init: only mu and nu are checked)."""
    mu, nu = wl.config_c1()
    bad = np.zeros_like(mu)
    bad[10, 17] = np.nan
    for dtype in (torch.float64, torch.float32):
        with pytest.raises(bfm.BFMError) as e:
            bfm.solve(cuda(mu, dtype), cuda(nu, dtype), phi_init=cuda(bad, dtype), max_iters=3)
        assert e.value.status == bfm.BFM_ENUMERIC
        assert "non-finite" in str(e.value)
    # the library stays usable afterwards
    r = bfm.solve(cuda(mu), cuda(nu), max_iters=3)
    assert np.isfinite(r.dual)


def _oracle_floor_hits(mu, nu, prm):
    """Runs the oracle and counts the step-rule updates whose result is
    sigma_min, by wrapping the oracle's own update function."""
    hits = [0]
    inner = ob.update_sigma

    def counting(sigma, increase, G, p):
        s = inner(sigma, increase, G, p)
        hits[0] += int(s == p.sigma_min)
        return s

    ob.update_sigma = counting
    try:
        o = ob.solve(mu, nu, prm)
    finally:
        ob.update_sigma = inner
    return o, hits[0]


@pytest.mark.parametrize("sigma0,sigma_min", [(0.0, 0.01), (40.0, 20.0), (5.0, 2.0)])
def test_sigma_floor_hits_match_oracle(sigma0, sigma_min):
    mu, nu = wl.config_c1()
    o, hits = _oracle_floor_hits(mu, nu, ob.Params(max_iters=20, sigma0=sigma0, sigma_min=sigma_min))
    plan = bfm.Plan(mu.shape, torch.float64, max_iters=20, sigma0=sigma0, sigma_min=sigma_min)
    r = plan.solve(cuda(mu), cuda(nu))
    lib_res = bfm.Result()
    assert hasattr(lib_res, "sigma_floor_hits")
    assert r.sigma_floor_hits == hits
    assert r.sigma == pytest.approx(o.sigma, rel=1e-12)
    if sigma_min > 1.0:
        assert hits > 0   # steps this large overshoot and are clamped


@pytest.mark.parametrize("shape", [(256, 256), (48, 36, 32)])
def test_deposit_grid_changes_only_the_order_of_sums(shape):
    """The deposition's workgroup count (set, or picked by
    bfm_autotune_deposit) changes only how the float64 partial sums are
    grouped (and the order of the float atomics): same iterations, same
    results to rounding."""
    rng = np.random.default_rng(8)
    mu = wl.random_gaussian_mixture(shape, 3, rng)
    nu = wl.random_gaussian_mixture(shape, 2, rng)
    base = bfm.Plan(shape, torch.float64, max_iters=8).solve(cuda(mu), cuda(nu))
    tuned = bfm.Plan(shape, torch.float64, max_iters=8)
    picked = tuned.autotune_deposit(base.phi, cuda(mu))
    tiles = int(np.prod([-(-n // t) for n, t in zip(shape, (16, 32) if len(shape) == 2 else (8, 8, 8))]))
    assert picked in (1024, 2048, 4096, 8192) or picked == -(-tiles // 8) * 8
    plans = [tuned]
    for G in (8, 1024, 8192):
        p = bfm.Plan(shape, torch.float64, max_iters=8)
        p.set_deposit_grid(G)
        plans.append(p)
    for p in plans:
        r = p.solve(cuda(mu), cuda(nu))
        assert r.iters == base.iters
        assert abs(r.dual - base.dual) <= 1e-11 * abs(base.dual)
        assert r.sigma == pytest.approx(base.sigma, rel=1e-12)
        assert float((r.phi - base.phi).abs().max()) <= 1e-9 * float(base.phi.abs().max())
