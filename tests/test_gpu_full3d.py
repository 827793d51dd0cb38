"""The 3D bench workload at its full size (c4: 384^3, 6-Gaussian mixtures,
float32), in the launch configuration the bench times: the c-transform at
sampled points against the definition over all 56.6M grid points, the
Poisson solve element by element against the oracle, and a few solve
iterations through properties that hold at any size."""
import numpy as np
import pytest
import torch

from oracle import bfm as ob
from paper_1905_12154_amd import bfm, workloads as wl

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
N3 = 384


def cuda(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def host(t):
    return t.detach().double().cpu().numpy()


def _axes(n):
    y = (np.arange(n) + 0.5) / n
    return y[:, None, None], y[None, :, None], y[None, None, :]


def _smooth3(n):
    x0, x1, x2 = _axes(n)
    return (0.2 * x0 ** 2 - 0.1 * x1 + 0.15 * x2 ** 2 + 0.05 * np.sin(7 * x0 * x2) * np.cos(3 * x1)).astype(np.float32)


def test_full_size_3d_ctransform_sampled():
    f = _smooth3(N3)
    got = host(bfm.ctransform(cuda(f)))
    y0, y1, y2 = _axes(N3)
    fd = f.astype(np.float64)
    rng = np.random.default_rng(2)
    for _ in range(6):
        i, j, k = rng.integers(0, N3, size=3)
        x = (np.array([i, j, k]) + 0.5) / N3
        ref = np.min(0.5 * ((x[0] - y0) ** 2 + (x[1] - y1) ** 2 + (x[2] - y2) ** 2) - fd)
        assert abs(got[i, j, k] - ref) <= 2e-6, (i, j, k)


def test_full_size_3d_poisson_matches_oracle():
    mu, nu = wl.config_c4()
    f = (nu - mu).astype(np.float32)
    g_t, G = bfm.poisson_neumann(cuda(f))
    gr, Gr = ob.poisson_neumann(f.astype(np.float64))
    assert np.max(np.abs(host(g_t) - gr)) <= 1e-4 * np.max(np.abs(gr))
    assert abs(G - Gr) <= 1e-4 * Gr


def test_full_size_3d_solve_properties():
    mu, nu = wl.config_c4()
    r = bfm.solve(cuda(mu), cuda(nu), max_iters=3)
    assert r.iters == 3
    assert abs(r.mass_mu - 1) < 1e-5 and abs(r.mass_nu - 1) < 1e-5
    T = host(r.T)
    assert T.min() >= 0.5 / N3 - 1e-7 and T.max() <= 1 - 0.5 / N3 + 1e-7
    phi = host(r.phi)
    psi = host(r.psi)
    y0, y1, y2 = _axes(N3)
    rng = np.random.default_rng(4)
    for _ in range(4):
        i, j, k = rng.integers(0, N3, size=3)
        x = (np.array([i, j, k]) + 0.5) / N3
        ref = np.min(0.5 * ((x[0] - y0) ** 2 + (x[1] - y1) ** 2 + (x[2] - y2) ** 2) - phi)
        assert abs(psi[i, j, k] - ref) <= 5e-6
    assert 0 < r.dual < 1.5 and r.G > 0
