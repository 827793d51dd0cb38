"""Batched solve of 2D quadratic-cost problems with one launch per pass over
all pairs (Algorithm 1 per pair; each pair keeps its own step size, gap and
stop flag): the form bfm_solve_batched takes when every pair is 2D with the
quadratic cost.  Checked against the plain solver run pair by pair (the
same iteration on every pair; deposition adds with float atomics, so the two
agree to rounding) and against the float64 oracle."""
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


def pairs(shapes, seed=0):
    rng = np.random.default_rng(seed)
    out = []
    for s in shapes:
        mu = wl.random_gaussian_mixture(s, int(rng.integers(2, 5)), rng)
        nu = wl.random_gaussian_mixture(s, int(rng.integers(2, 5)), rng)
        out.append((mu, nu))
    return out


# ragged sizes, odd line counts (27 = 3^3), lines of 4..1024 points
SHAPES = [(64, 64), (96, 48), (128, 128), (48, 64), (27, 48), (384, 256), (256, 384), (1024, 128), (12, 8),
          (64, 64)]


def _compare(rb, mus, nus, iters, dtype, **kw):
    """float64: everything to rounding.  float32: the scalars and potentials
    to a few hundred ulps; the map in grid cells, where the two forms differ
    by more (the batched form runs the rows of a c-transform before its
    columns, the plain float32 form the columns first, and the map's central
    difference multiplies a potential difference by n / 2)."""
    tol = 1e-10 if dtype == torch.float64 else 2e-5
    for i, (m, n) in enumerate(zip(mus, nus)):
        rp = bfm.solve(m, n, max_iters=iters, return_map=True, **kw)
        assert (rb[i].iters, rb[i].converged) == (rp.iters, rp.converged), i
        assert abs(rb[i].dual - rp.dual) <= tol * max(1.0, abs(rp.dual)), i
        assert abs(rb[i].gap - rp.gap) <= tol * max(1e-2, rp.gap) * 10, i
        assert rb[i].sigma == pytest.approx(rp.sigma, rel=1e-12 if dtype == torch.float64 else 1e-5), i
        assert rb[i].sigma_floor_hits == rp.sigma_floor_hits, i
        for a, b in ((rb[i].phi, rp.phi), (rb[i].psi, rp.psi)):
            assert float((a - b).abs().max()) <= tol * max(1.0, float(b.abs().max())) * 10, i
        cells = torch.stack([(rb[i].T[a] - rp.T[a]).abs() * m.shape[a] for a in range(2)]).amax(0).flatten().double()
        if dtype == torch.float64:
            assert float(cells.max()) <= 1e-8, i
        else:
            # T is a central difference of phi^c: a difference d in phi^c
            # moves T by about n d / 2, which is n^2 d / 2 cells.  Two float32
            # runs of one problem, batched or plain, differ in phi^c by up to
            # ~1e-5 after a few iterations, since the deposition's float
            # atomics add in a different order in every run (measured: two
            # plain runs of a 1024^2 pair differ by up to 2 cells after six
            # iterations, on 99% of the cells by under 0.1).  Bars: 1e-5 n^2
            # cells at most, a quarter cell on 99% of the cells.
            n = max(m.shape)
            assert float(cells.max()) <= 1e-5 * n * n, i
            assert float(torch.quantile(cells.float(), 0.99)) <= 0.25, i


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("iters,K", [(20, 8), (5, 8), (0, 4), (9, 1), (13, 4)])
def test_multi_batched_equals_plain(dtype, iters, K):
    ps = pairs(SHAPES)
    mus = [cuda(m, dtype) for m, _ in ps]
    nus = [cuda(n, dtype) for _, n in ps]
    rb = bfm.solve_batched(mus, nus, max_iters=iters, iters_per_graph=K, return_map=True)
    _compare(rb, mus, nus, iters, dtype)


def test_multi_batched_against_oracle():
    ps = pairs([(48, 64), (96, 48), (27, 48)], seed=5)
    rb = bfm.solve_batched([cuda(m) for m, _ in ps], [cuda(n) for _, n in ps], max_iters=10, iters_per_graph=4,
                           return_map=True)
    for (m, n), r in zip(ps, rb):
        o = ob.solve(m, n, ob.Params(max_iters=10))
        assert abs(r.dual - o.dual) <= 1e-10
        assert abs(r.w2sq - o.w2sq) <= 1e-5 * o.w2sq
        assert r.sigma == pytest.approx(o.sigma, rel=1e-12)
        assert np.max(np.abs(host(r.phi) - o.phi)) <= 1e-7
        for a in range(2):
            assert np.max(np.abs(host(r.T[a]) - o.T[a])) * m.shape[a] <= 1e-3


def test_multi_batched_stop_flags_per_pair():
    # the two discs converge early, the Gaussian pairs later or not at all
    d_mu, d_nu = wl.two_discs(64)
    rest = pairs([(64, 64), (128, 64)], seed=3)
    mus = [cuda(d_mu)] + [cuda(m) for m, _ in rest]
    nus = [cuda(d_nu)] + [cuda(n) for _, n in rest]
    rb = bfm.solve_batched(mus, nus, max_iters=40, tol=2e-5, iters_per_graph=4, return_map=True)
    _compare(rb, mus, nus, 40, torch.float64, tol=2e-5)
    assert rb[0].converged and rb[0].iters < 40


def test_multi_batched_more_pairs_than_one_launch_holds():
    # 70 pairs: two chunks of pairs, each with its own table
    rng = np.random.default_rng(17)
    shapes = [tuple(int(x) for x in rng.choice([16, 24, 32, 48], size=2)) for _ in range(70)]
    ps = pairs(shapes, seed=11)
    mus = [cuda(m) for m, _ in ps]
    nus = [cuda(n) for _, n in ps]
    rb = bfm.solve_batched(mus, nus, max_iters=6, iters_per_graph=2, return_map=True)
    _compare(rb, mus, nus, 6, torch.float64)


def test_multi_batched_c5_pairs_f32():
    """float32 on the first six pairs of the 64-pair workload (128^2 to
    1024^2).  Six iterations: later, where J changes by little more than the
    float32 rounding of the fields moves it, the step rule's comparison of
    J_new - J_old can come out differently in two runs of the same problem
    (the deposition's float atomics add in a different order each run), and
    the two runs then follow different step sizes."""
    sides = wl.c5_sides()
    ps = [wl.config_c5_pair(i, sides[i]) for i in range(6)]
    mus = [cuda(m, torch.float32) for m, _ in ps]
    nus = [cuda(n, torch.float32) for _, n in ps]
    rb = bfm.solve_batched(mus, nus, max_iters=6, iters_per_graph=2, return_map=True)
    _compare(rb, mus, nus, 6, torch.float32)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_grad_batched_equals_per_pair_grad(dtype):
    """bfm_grad_batched (three launches for the batch) against bfm_grad per
    pair on the same potentials: the same formula, means summed in another
    order, so equal to rounding."""
    ps = pairs([(64, 64), (96, 48), (27, 48), (24, 16, 12), (128, 128)], seed=4)
    plans, phis, psis = [], [], []
    for m, n in ps:
        r = bfm.solve(cuda(m, dtype), cuda(n, dtype), max_iters=5)
        plans.append(bfm.plan_for(m.shape, dtype))
        phis.append(r.phi)
        psis.append(r.psi)
    scales = [1.0, -2.0, 0.5, 3.0, 1.25]
    ws = bfm._aligned_workspaces(plans, DEV)
    gmus, gnus = bfm.grad_batched(plans, phis, psis, scales, ws)
    tol = 1e-12 if dtype == torch.float64 else 1e-6
    for i in range(len(ps)):
        a, b = plans[i].grad(phis[i], psis[i], scales[i])
        assert float((gmus[i] - a).abs().max()) <= tol * float(a.abs().max())
        assert float((gnus[i] - b).abs().max()) <= tol * float(b.abs().max())
        assert abs(float(gmus[i].double().sum())) <= 1e-6 * float(gmus[i].double().abs().sum())


def test_multi_batched_compaction_matches_plain():
    """70 pairs over two chunks whose stop iterations spread from 2 to 40
    (the float64 oracle gives 40 of them stopped by iteration 4 at this
    tolerance): after the replay where at most half are still running, the
    tables are rebuilt over the running pairs alone (one chunk) and the graph
    is captured again.  Every pair must still match its own plain solve."""
    rng = np.random.default_rng(23)
    shapes = [tuple(int(x) for x in rng.choice([16, 24, 32, 48, 64], size=2)) for _ in range(70)]
    ps = pairs(shapes, seed=29)
    mus = [cuda(m) for m, _ in ps]
    nus = [cuda(n) for _, n in ps]
    rb = bfm.solve_batched(mus, nus, max_iters=40, tol=1e-3, iters_per_graph=2, return_map=True)
    _compare(rb, mus, nus, 40, torch.float64, tol=1e-3)
    its = sorted(r.iters for r in rb)
    assert its[35] <= 6 and its[-1] == 40, its
