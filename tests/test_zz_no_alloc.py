"""bfm_solve_noalloc (the solve's scratch in the library's static device
array, no allocation) against bfm_solve with a caller workspace, both called
through the C ABI: two calls in a row, the second on a smaller grid; then a
converged run followed by a run that must start from a fresh state.

Deposition adds with float atomics whose order varies between runs, so the
two entry points agree to rounding (float64: 1e-12 relative on the scalars,
1e-10 of the field scale on the fields), not bitwise."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1905_12154_amd import bfm, workloads as wl

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def cuda(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def _vp(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream(torch.device(DEV)).cuda_stream)


def _outputs(plan, like):
    return (torch.empty_like(like), torch.empty_like(like),
            torch.empty((len(plan.shape),) + plan.shape, dtype=plan.dtype, device=DEV))


def _run_noalloc(plan, mu, nu):
    phi, psi, T = _outputs(plan, mu)
    res = bfm.Result()
    st = bfm.lib().bfm_solve_noalloc(plan.handle, _vp(mu), _vp(nu), None, _vp(phi), _vp(psi), _vp(T), _stream(),
                                     ctypes.byref(res))
    assert st == bfm.BFM_OK, bfm.lib().bfm_last_error().decode()
    return phi, psi, T, res


def _run_workspace(plan, mu, nu):
    phi, psi, T = _outputs(plan, mu)
    ws = torch.empty(plan.ws_bytes + 256, dtype=torch.uint8, device=DEV)
    off = (-ws.data_ptr()) % 256
    ws = ws[off:off + plan.ws_bytes]
    res = bfm.Result()
    st = bfm.lib().bfm_solve(plan.handle, _vp(mu), _vp(nu), None, _vp(phi), _vp(psi), _vp(T), _vp(ws),
                             plan.ws_bytes, _stream(), ctypes.byref(res))
    assert st == bfm.BFM_OK, bfm.lib().bfm_last_error().decode()
    return phi, psi, T, res


def _same(a, b, dtype):
    fr = 1e-10 if dtype == torch.float64 else 2e-5
    sr = 1e-12 if dtype == torch.float64 else 1e-6
    (pa, sa, Ta, ra), (pb, sb, Tb, rb) = a, b
    assert (ra.iters, ra.converged, ra.status) == (rb.iters, rb.converged, rb.status)
    assert abs(ra.dual - rb.dual) <= sr * abs(rb.dual)
    assert abs(ra.primal - rb.primal) <= sr * abs(rb.primal)
    assert ra.sigma == pytest.approx(rb.sigma, rel=sr)
    assert ra.sigma_floor_hits == rb.sigma_floor_hits
    for x, y in ((pa, pb), (sa, sb), (Ta, Tb)):
        assert float((x - y).abs().max()) <= fr * max(1.0, float(y.abs().max()))


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_noalloc_matches_workspace_solve_twice(dtype):
    big = wl.config_c1()
    rng = np.random.default_rng(3)
    small = (wl.random_gaussian_mixture((48, 32), 2, rng), wl.random_gaussian_mixture((48, 32), 3, rng))
    for mu, nu in (big, small):
        plan = bfm.Plan(mu.shape, dtype, max_iters=15)
        tmu, tnu = cuda(mu, dtype), cuda(nu, dtype)
        got = _run_noalloc(plan, tmu, tnu)
        ref = _run_workspace(plan, tmu, tnu)
        _same(got, ref, dtype)


def test_noalloc_fresh_state_after_a_converged_call():
    # the first call stops early and leaves its stop flag set in the static
    # array; the second (smaller) call must start from a fresh state
    d_mu, d_nu = wl.two_discs(64)
    p1 = bfm.Plan(d_mu.shape, torch.float64, max_iters=40, tol=2e-5)
    r1 = _run_noalloc(p1, cuda(d_mu), cuda(d_nu))[3]
    assert r1.converged and r1.iters < 40
    rng = np.random.default_rng(8)
    mu, nu = wl.random_gaussian_mixture((32, 48), 3, rng), wl.random_gaussian_mixture((32, 48), 2, rng)
    p2 = bfm.Plan(mu.shape, torch.float64, max_iters=10)
    got = _run_noalloc(p2, cuda(mu), cuda(nu))
    ref = _run_workspace(p2, cuda(mu), cuda(nu))
    assert got[3].iters == 10
    _same(got, ref, torch.float64)
