"""HIP path versus the CPU float64 oracle, element by element on seeded inputs.

Tolerances: float64 kernels agree with the oracle to rounding (1e-12 or
tighter relative); float32 kernels to a few hundred float32 ulps of the
field's scale.  The whole solve at the parity configuration (64^2, float64,
60 iterations) must give W2^2 within 1e-5 relative and the map within 1e-3
grid cells.
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


def rand_field(shape, seed, kind="normal"):
    rng = np.random.default_rng(seed)
    if kind == "normal":
        return rng.normal(scale=0.2, size=shape)
    if kind == "cconcave":   # a c-transform output: many collinear hull runs and ties
        return ob.ctransform(rng.normal(scale=0.3, size=shape))
    if kind == "steps":      # piecewise-constant jumps: long pops across lanes
        f = np.zeros(shape)
        for a in range(len(shape)):
            idx = np.arange(shape[a]).reshape([-1 if b == a else 1 for b in range(len(shape))])
            f = f + 0.3 * ((idx * 7 // shape[a]) % 2)
        return f + 0.01 * rng.normal(size=shape)
    if kind == "potential":  # smooth potential plus a step of a gradient ascent
        xs = ob.centres(shape)
        f = sum(0.3 * x * x - 0.2 * x for x in xs) + 0.05 * np.sin(7 * xs[0])
        return f + 0.02 * rng.normal(size=shape)
    raise ValueError(kind)


CT_SHAPES = [(4, 4), (6, 12), (64, 64), (96, 48), (48, 384), (128, 256), (1024, 8), (4096, 4),
             (8, 6, 4), (24, 32, 18), (12, 96, 16)]


@pytest.mark.parametrize("shape", CT_SHAPES)
@pytest.mark.parametrize("kind", ["normal", "cconcave", "steps", "potential"])
def test_ctransform_f64_matches_definition(shape, kind):
    f = rand_field(shape, 1, kind)
    got = host(bfm.ctransform(cuda(f)))
    ref = ob.ctransform(f)
    assert np.max(np.abs(got - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("shape", [(64, 64), (96, 48), (384, 128), (1024, 16), (24, 32, 18)])
@pytest.mark.parametrize("kind", ["normal", "cconcave", "potential"])
def test_ctransform_f32(shape, kind):
    f = rand_field(shape, 2, kind)
    f32 = f.astype(np.float32).astype(np.float64)
    got = host(bfm.ctransform(cuda(f32, torch.float32)))
    ref = ob.ctransform(f32)
    scale = max(1.0, np.max(np.abs(ref)))
    assert np.max(np.abs(got - ref)) <= 300 * np.finfo(np.float32).eps * scale


def _ct_modes(shape, esz):
    """Every launch mode that applies to a shape: points per lane, lines per
    workgroup on strided axes, one group per workgroup (1) or persistent (2)."""
    def four_lines_fit(n, C, esz):   # LDS of a four-line group within the 150 KB budget
        tpl = 1 << int(np.ceil(np.log2(max(1, -(-n // C)))))
        npad = n + n // 16 + 1
        return ((4 * npad * esz + 8 * npad * 2 + 3) & ~3) + 32 * tpl <= 150 * 1024

    out = []
    for C in (4, 8, 12, 16):
        if any(C * 1024 < n for n in shape):
            continue
        for lpb in (1, 2, 4):
            for pers in (1, 2):
                # persistent: rows need n % 4 == 0; a strided axis needs a group of
                # four lines (inner % 4 == 0, LDS room, >= 16 lanes per line)
                ok = shape[-1] % 4 == 0 and all(
                    lpb == 4 and int(np.prod(shape[a + 1:])) % 4 == 0 and four_lines_fit(shape[a], C, esz)
                    and -(-shape[a] // C) > 8 for a in range(len(shape) - 1))
                # True: must run; False: must be rejected; None: either (the
                # launch shape may widen a group to whole waves)
                if lpb == 2:   # two-line groups: rely on the persistent kernel's own checks
                    ok = False
                out.append(((C, lpb, pers), True if pers == 1 or ok else (False if shape[-1] % 4 else None)))
    return out


@pytest.mark.parametrize("shape", [(64, 64), (96, 48), (6, 12), (24, 36), (16, 54), (384, 128), (1024, 8),
                                   (24, 32, 18), (8, 12, 24), (4096, 16)])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_ctransform_every_launch_mode(shape, dtype):
    """Each c-transform kernel variant (including the persistent prefetching
    one, with its wave-level merge synchronisation) against the definition."""
    f = rand_field(shape, 3, "potential")
    if dtype == torch.float32:
        f = f.astype(np.float32).astype(np.float64)
    ref = ob.ctransform(f)
    tol = (1e-13 if dtype == torch.float64 else 300 * np.finfo(np.float32).eps) * max(1.0, np.max(np.abs(ref)))
    plan = bfm.Plan(shape, dtype)
    for mode, applies in _ct_modes(shape, 8 if dtype == torch.float64 else 4):
        plan.set_tuning([mode] * len(shape))
        assert plan.tuning() == [mode] * len(shape)
        if applies is False:
            with pytest.raises(bfm.BFMError):
                plan.ctransform(cuda(f, dtype))
            continue
        try:
            got = host(plan.ctransform(cuda(f, dtype)))
        except bfm.BFMError:
            assert applies is None, mode
            continue
        assert np.max(np.abs(got - ref)) <= tol, mode


def test_set_tuning_rejects_bad_values():
    plan = bfm.Plan((64, 4096), torch.float32)
    for bad in ([(6, 0, 0), (0, 0, 0)], [(12, 0, 0), (6000, 0, 0)], [(8, 3, 0), (0, 0, 0)],
                [(8, 4, 3), (0, 0, 0)], [(0, 0, 0), (2, 0, 0)]):
        with pytest.raises(bfm.BFMError) as e:
            plan.set_tuning(bad)
        assert e.value.status == bfm.BFM_EINVAL
    assert plan.tuning() == [(0, 0, 0), (0, 0, 0)]


def _blocked(x):
    """Column-blocked layout of a 2D array: element (r, c) at (c // 4) 4 R + 4 r + c % 4."""
    R, K = x.shape
    return np.ascontiguousarray(x.reshape(R, K // 4, 4).transpose(1, 0, 2)).reshape(R, K)


@pytest.mark.parametrize("shape,dtype,tuning", [((256, 512), torch.float32, None),
                                                ((4096, 16), torch.float32, None),
                                                ((96, 36), torch.float32, [(8, 4, 2), (16, 0, 2)]),
                                                ((128, 64), torch.float64, [(8, 4, 2), (8, 0, 2)])])
def test_ctransform_blocked_passes(shape, dtype, tuning):
    """The two passes of the column-blocked 2D transform: pass 0 is the
    column pass of -f in the blocked layout, pass 1 the row pass back to
    row-major; with a weight, pass 1 also returns sum(out * weight)."""
    f = rand_field(shape, 4, "potential")
    if dtype == torch.float32:
        f = f.astype(np.float32).astype(np.float64)
    plan = bfm.Plan(shape, dtype)
    if tuning is not None:
        plan.set_tuning(tuning)
    tol = (1e-13 if dtype == torch.float64 else 300 * np.finfo(np.float32).eps)
    mid = plan.ctransform_pass(cuda(f, dtype), 0)
    ref_mid = _blocked(ob.line_min(-f, 0))
    assert np.max(np.abs(host(mid) - ref_mid)) <= tol * max(1.0, np.max(np.abs(ref_mid)))
    w = np.random.default_rng(5).uniform(0.0, 2.0, size=shape)
    out, total = plan.ctransform_pass(mid, 1, weight=cuda(w, dtype), want_sum=True)
    ref = ob.ctransform(f)
    assert np.max(np.abs(host(out) - ref)) <= tol * max(1.0, np.max(np.abs(ref)))
    exact = float(np.sum(host(out) * host(cuda(w, dtype))))
    assert abs(total - exact) <= 1e-12 * np.sum(np.abs(host(out)) * w) + 1e-300
    assert np.array_equal(host(plan.ctransform_pass(mid, 1)), host(out))   # same kernel without the sum


def test_ctransform_pass_errors():
    f64 = bfm.Plan((64, 64), torch.float64)          # default float64 shapes are not persistent
    x = cuda(np.zeros((64, 64)))
    with pytest.raises(bfm.BFMError) as e:
        f64.ctransform_pass(x, 0)
    assert e.value.status == bfm.BFM_EUNSUPPORTED
    odd = bfm.Plan((64, 54), torch.float32)           # rows not a multiple of 4
    with pytest.raises(bfm.BFMError) as e:
        odd.ctransform_pass(cuda(np.zeros((64, 54)), torch.float32), 0)
    assert e.value.status == bfm.BFM_EUNSUPPORTED
    p3 = bfm.Plan((16, 16, 16), torch.float32)
    with pytest.raises(bfm.BFMError) as e:
        p3.ctransform_pass(cuda(np.zeros((16, 16, 16)), torch.float32), 0)
    assert e.value.status == bfm.BFM_EUNSUPPORTED
    ok = bfm.Plan((64, 64), torch.float32)
    y = cuda(np.zeros((64, 64)), torch.float32)
    for bad in (lambda: ok.ctransform_pass(y, 2), lambda: ok.ctransform_pass(y, 0, out=y)):
        with pytest.raises(bfm.BFMError) as e:
            bad()
        assert e.value.status == bfm.BFM_EINVAL


def test_ctransform_in_place_and_linear_closed_form():
    shape = (96, 128)
    xs = ob.centres(shape)
    a = (5 / 96, -7 / 128)
    f = a[0] * xs[0] + a[1] * xs[1] + np.zeros(shape)
    t = cuda(f)
    out = bfm.plan_for(shape, torch.float64).ctransform(t, out=t)   # in place
    ref = ob.ctransform(f)
    assert np.max(np.abs(host(out) - ref)) <= 1e-14


# (9, 12), (27, 16), (9, 27, 8): an odd number of contiguous lines, so the last
# pair of lines has no second line
@pytest.mark.parametrize("shape", [(64, 64), (96, 384), (6, 4), (24, 32, 18), (4096, 16), (9, 12), (27, 16),
                                   (9, 27, 8)])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_poisson_matches_oracle(shape, dtype):
    f = np.random.default_rng(3).normal(size=shape)
    f = f.astype(np.float32).astype(np.float64) if dtype == torch.float32 else f
    g, G = bfm.poisson_neumann(cuda(f, dtype))
    gr, Gr = ob.poisson_neumann(f)
    # FFT roundoff (~eps log2 n |f|) amplified by 1/lambda on the low modes
    tol = 1e-11 if dtype == torch.float64 else 2e-5
    assert np.max(np.abs(host(g) - gr)) <= tol * np.max(np.abs(gr))
    assert abs(G - Gr) <= tol * abs(Gr) * 10


def _potential_map_case(shape, seed):
    rng = np.random.default_rng(seed)
    xs = ob.centres(shape)
    pc = sum(-0.15 * x * x + 0.05 * x for x in xs) + 0.004 * rng.normal(size=shape)
    mass = rng.uniform(0.0, 2.0, size=shape)
    mass[rng.uniform(size=shape) < 0.3] = 0.0
    return pc, mass


@pytest.mark.parametrize("shape", [(64, 64), (96, 384), (4, 6), (24, 32, 18), (512, 512)])
def test_pushforward_f64_matches_oracle(shape):
    pc, mass = _potential_map_case(shape, 5)
    rho, T, P = bfm.pushforward(cuda(pc), cuda(mass))
    Tr = ob.transport_map(pc)
    rr = ob.pushforward(mass, Tr)
    Pr = ob.primal_cost(mass, Tr)
    for a in range(len(shape)):
        assert np.max(np.abs(host(T[a]) - Tr[a])) <= 1e-13
    assert np.max(np.abs(host(rho) - rr)) <= 1e-12 * np.max(rr)
    assert abs(P - Pr) <= 1e-12 * abs(Pr)


def test_pushforward_f32_mass_and_parity():
    shape = (256, 384)
    pc, mass = _potential_map_case(shape, 6)
    pc32 = pc.astype(np.float32).astype(np.float64)
    m32 = mass.astype(np.float32).astype(np.float64)
    rho, T, P = bfm.pushforward(cuda(pc32, torch.float32), cuda(m32, torch.float32))
    rr = ob.pushforward(m32, ob.transport_map(pc32))
    assert abs(host(rho).sum() - m32.sum()) <= 1e-6 * m32.sum()
    assert np.max(np.abs(host(rho) - rr)) <= 1e-4 * np.max(rr)


# ----------------------------------------------------------------- solve

def _solve_both(mu, nu, dtype, iters, **kw):
    r = bfm.solve(cuda(mu, dtype), cuda(nu, dtype), max_iters=iters, **kw)
    o = ob.solve(mu, nu, ob.Params(max_iters=iters, **kw))
    return r, o


def test_solve_parity_c1_f64():
    """Parity configuration: 64^2, 3-Gaussian mixtures, float64, 60 iterations."""
    mu, nu = wl.config_c1()
    r, o = _solve_both(mu, nu, torch.float64, 60)
    assert r.iters == o.iters == 60
    assert abs(r.w2sq - o.w2sq) <= 1e-5 * abs(o.w2sq)
    n = mu.shape[0]
    for a in range(2):
        assert np.max(np.abs(host(r.T[a]) - o.T[a])) * n <= 1e-3
    # potentials, mean-normalised (full support: unique up to the constant)
    assert np.max(np.abs(host(r.phi) - o.phi)) <= 1e-6
    assert np.max(np.abs(host(r.psi) - o.psi)) <= 1e-6
    assert abs(r.gap - o.gap) <= 1e-6 + 1e-5 * o.gap
    assert r.sigma == pytest.approx(o.sigma, rel=1e-12)


def test_solve_trace_matches_oracle_first_iterations():
    mu, nu = wl.config_c1()
    r, o = _solve_both(mu, nu, torch.float64, 6)
    assert abs(r.dual - o.dual) <= 1e-11
    assert abs(r.G - o.G) <= 1e-11 * max(1.0, o.G)
    assert abs(r.primal - o.primal) <= 1e-11


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-12), (torch.float32, 2e-6)])
def test_two_discs_exact_cost(dtype, tol):
    mu, nu = wl.two_discs(128)
    r = bfm.solve(cuda(mu, dtype), cuda(nu, dtype), max_iters=10)
    assert abs(r.dual - 0.25) <= tol


def test_stop_rule_same_iteration_as_oracle():
    mu, nu = wl.two_discs(128)
    r, o = _solve_both(mu, nu, torch.float64, 30, tol=1e-5)
    assert r.converged and o.converged
    assert r.iters == o.iters < 30
    assert abs(r.gap - o.gap) <= 1e-10
    assert abs(r.dual - 0.25) <= 1e-12


def test_square_to_four_exact_dual_with_gap_floor():
    # discontinuous map: the dual reaches 1/16 while |P - D| keeps an O(h)
    # floor, so a tolerance below it is never met (converged = False)
    mu, nu = wl.square_to_four(128)
    r, o = _solve_both(mu, nu, torch.float64, 12, tol=1e-4)
    assert not r.converged and not o.converged and r.iters == o.iters == 12
    assert abs(r.dual - 1 / 16) <= 1e-12
    assert abs(r.gap - o.gap) <= 1e-9


@pytest.mark.parametrize("shape", [(96, 384), (48, 64), (27, 48)])
def test_solve_parity_rectangular(shape):
    rng = np.random.default_rng(9)
    mu = wl.random_gaussian_mixture(shape, 3, rng)
    nu = wl.random_gaussian_mixture(shape, 2, rng)
    r, o = _solve_both(mu, nu, torch.float64, 12)
    assert abs(r.dual - o.dual) <= 1e-10
    for a in range(2):
        assert np.max(np.abs(host(r.T[a]) - o.T[a])) * shape[a] <= 1e-3


def test_solve_parity_3d_f64():
    mu, nu = wl.two_balls(32)
    r, o = _solve_both(mu, nu, torch.float64, 8)
    assert abs(r.dual - o.dual) <= 1e-10
    rng = np.random.default_rng(4)
    shape = (16, 24, 18)
    mu = wl.random_gaussian_mixture(shape, 2, rng)
    nu = wl.random_gaussian_mixture(shape, 3, rng)
    r, o = _solve_both(mu, nu, torch.float64, 8)
    assert abs(r.dual - o.dual) <= 1e-10
    for a in range(3):
        assert np.max(np.abs(host(r.T[a]) - o.T[a])) * shape[a] <= 1e-3


def test_solve_f32_error_vs_oracle_c1():
    """float32 fields with float64 sums: error against the float64 oracle."""
    mu, nu = wl.config_c1()
    r = bfm.solve(cuda(mu, torch.float32), cuda(nu, torch.float32), max_iters=60)
    o = ob.solve(mu, nu, ob.Params(max_iters=60))
    assert abs(r.w2sq - o.w2sq) <= 1e-4 * o.w2sq
    for a in range(2):
        assert np.max(np.abs(host(r.T[a]) - o.T[a])) * 64 <= 0.05


def test_max_iters_zero_and_warm_start():
    mu, nu = wl.config_c1()
    r0 = bfm.solve(cuda(mu), cuda(nu), max_iters=0)
    assert r0.iters == 0 and r0.dual == 0.0
    r1 = bfm.solve(cuda(mu), cuda(nu), max_iters=10)
    # resume from the returned potential: the head of the warm start is the
    # state the first run ended at
    r2 = bfm.solve(cuda(mu), cuda(nu), max_iters=0, phi_init=r1.phi)
    assert abs(r2.dual - r1.dual) <= 1e-13


@pytest.mark.parametrize("bad", ["negative", "nan", "mass"])
def test_invalid_density_rejected(bad):
    mu, nu = wl.config_c1()
    mu = mu.copy()
    if bad == "negative":
        mu[3, 3] = -1.0
    elif bad == "nan":
        mu[5, 7] = np.nan
    else:
        mu = mu * 1.01
    with pytest.raises(bfm.BFMError) as e:
        bfm.solve(cuda(mu), cuda(nu), max_iters=2)
    assert e.value.status == bfm.BFM_EINVAL


# ------------------------------------------------ full size (4096^2, float32)

@pytest.fixture(scope="module")
def c3():
    return wl.config_c3()


def test_full_size_ctransform_sampled(c3):
    """c-transform at 4096^2 in the launch configuration of the solver,
    checked at sampled points against the definition over all 16.7M y."""
    mu, _ = c3
    n = mu.shape[0]
    xs = ob.centres(mu.shape)
    f = (0.2 * xs[0] ** 2 - 0.1 * xs[1] + 0.05 * np.sin(9 * xs[0] * xs[1])).astype(np.float32)
    got = host(bfm.ctransform(cuda(f, torch.float32)))
    y0 = ((np.arange(n) + 0.5) / n)[:, None]
    y1 = ((np.arange(n) + 0.5) / n)[None, :]
    fd = f.astype(np.float64)
    rng = np.random.default_rng(0)
    for _ in range(24):
        i, j = rng.integers(0, n, size=2)
        x0, x1 = (i + 0.5) / n, (j + 0.5) / n
        ref = np.min(0.5 * ((x0 - y0) ** 2 + (x1 - y1) ** 2) - fd)
        assert abs(got[i, j] - ref) <= 2e-6, (i, j)


def test_full_size_pushforward_and_poisson(c3):
    mu, nu = c3
    mu32 = mu.astype(np.float32)
    xs = ob.centres(mu.shape)
    pc = (-0.1 * xs[0] ** 2 - 0.05 * xs[1] + 0.02 * np.cos(5 * xs[1]) + np.zeros(mu.shape)).astype(np.float32)
    rho, T, P = bfm.pushforward(cuda(pc, torch.float32), cuda(mu32, torch.float32))
    rr = ob.pushforward(mu32.astype(np.float64), ob.transport_map(pc.astype(np.float64)))
    rh = host(rho)
    assert abs(rh.sum() - mu32.astype(np.float64).sum()) <= 1e-5 * mu32.sum()
    assert np.max(np.abs(rh - rr)) <= 1e-3 * rr.max()
    f = (nu - rr).astype(np.float32)
    g, G = bfm.poisson_neumann(cuda(f, torch.float32))
    gr, Gr = ob.poisson_neumann(f.astype(np.float64))
    assert np.max(np.abs(host(g) - gr)) <= 1e-4 * np.max(np.abs(gr))
    assert abs(G - Gr) <= 1e-4 * Gr


def test_full_size_solve_properties(c3):
    """A few iterations of the 4096^2 float32 solve: mass, c-conjugacy of the
    returned pair at sampled points, map inside the box, dual below primal."""
    mu, nu = c3
    r = bfm.solve(cuda(mu, torch.float32), cuda(nu, torch.float32), max_iters=3)
    assert r.iters == 3
    assert abs(r.mass_mu - 1) < 1e-5 and abs(r.mass_nu - 1) < 1e-5
    n = mu.shape[0]
    T = host(r.T)
    assert T.min() >= 0.5 / n - 1e-7 and T.max() <= 1 - 0.5 / n + 1e-7
    phi = host(r.phi)
    psi = host(r.psi)
    y0 = ((np.arange(n) + 0.5) / n)[:, None]
    y1 = ((np.arange(n) + 0.5) / n)[None, :]
    rng = np.random.default_rng(1)
    for _ in range(12):
        i, j = rng.integers(0, n, size=2)
        x0, x1 = (i + 0.5) / n, (j + 0.5) / n
        ref = np.min(0.5 * ((x0 - y0) ** 2 + (x1 - y1) ** 2) - phi)
        assert abs(psi[i, j] - ref) <= 5e-6
    assert 0 < r.dual < 0.5
