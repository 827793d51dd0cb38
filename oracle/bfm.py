"""CPU float64 oracle of the back-and-forth method (quadratic cost, uniform grid).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  It shares no code
with the HIP path and imports nothing from the product package.

Everything here follows the paper (Jacobs & Leger, "A fast approach to optimal
transport: the back-and-forth method"):

* grid: Omega = [0,1]^d discretised by a regular grid (Section 4.3); cells are
  centred, x_i = (i + 1/2) h_a on axis a, and densities are grid values with
  cell_volume * sum = 1;
* c-transform: its definition (Section 2.1), f^c(x) = min_y 1/2|x-y|^2 - f(y)
  over grid points y, evaluated axis by axis through the separable
  decomposition of Section 4.1 -- each one-dimensional step is a plain
  minimum over every point of the line (C helper ``line_min.c``);
* map: T(x) = x - grad f^c(x) (Lemma on c-transform properties, (ii), with
  h = |.|^2/2), gradient by central differences, one-sided at the faces,
  clamped to the box of cell centres;
* pushforward: the test-function definition of T#mu (Section 2.1) taken with
  piecewise-bilinear (trilinear) test functions, i.e. cloud-in-cell
  deposition of each cell's mass at T(x);
* H^1 gradient: (-Laplacian)^{-1} of the mean-free first variation with zero
  Neumann data (H^1-gradient lemma, eq. gradients_J_I), the Laplacian being
  the standard second-difference stencil whose eigenbasis is the DCT-II
  (scipy's DCT is used as the library transform);
* dual functionals J and I (eq. defJ / defI) as cell-volume weighted sums;
* Algorithm 1 (back-and-forth iteration) with the step-size rule of
  Section 4.2 (beta1=1/4, beta2=3/4, alpha1=5/4, alpha2=4/5,
  sigma0 = 8 min(1/max mu, 1/max nu), floor sigma_min = 0.01, no backtracking).
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np
import scipy.fft

from . import _native

WORKERS = os.cpu_count() or 1


# ---------------------------------------------------------------------------
# grid
# ---------------------------------------------------------------------------

def spacing(shape: Sequence[int]) -> List[float]:
    return [1.0 / n for n in shape]


def cell_vol(shape: Sequence[int]) -> float:
    v = 1.0
    for n in shape:
        v /= n
    return v


def centres(shape: Sequence[int]) -> List[np.ndarray]:
    """x_a = (i_a + 1/2) h_a as arrays broadcastable to ``shape``."""
    d = len(shape)
    out = []
    for a, n in enumerate(shape):
        s = [1] * d
        s[a] = n
        out.append(((np.arange(n, dtype=np.float64) + 0.5) / n).reshape(s))
    return out


# ---------------------------------------------------------------------------
# c-transform (Definition of the c-transform; separable form, Section 4.1)
# ---------------------------------------------------------------------------

def line_min(u: np.ndarray, axis: int) -> np.ndarray:
    """M_a[u](x) = min over y on the line through x along ``axis`` of
    1/2 (x_a - y_a)^2 + u(y)  -- one-dimensional c-transform step."""
    n = u.shape[axis]
    v = np.ascontiguousarray(np.moveaxis(np.asarray(u, dtype=np.float64), axis, -1))
    out = np.empty_like(v)
    _native.lib().oracle_line_min(v.ctypes.data, out.ctypes.data, v.size // n, n, 1.0 / n)
    return np.moveaxis(out, -1, axis)


def line_min_p(u: np.ndarray, axis: int, p: float) -> np.ndarray:
    """min over y on the line through x along ``axis`` of |x_a - y_a|^p / p + u(y)
    (the one-dimensional step for the power cost of eq. p_costs)."""
    n = u.shape[axis]
    v = np.ascontiguousarray(np.moveaxis(np.asarray(u, dtype=np.float64), axis, -1))
    out = np.empty_like(v)
    _native.lib().oracle_line_min_p(v.ctypes.data, out.ctypes.data, v.size // n, n, 1.0 / n, float(p))
    return np.moveaxis(out, -1, axis)


def _powers(ndim: int, powers) -> List[float]:
    """Per-axis exponents of the separable cost sum_a |x_a - y_a|^{p_a} / p_a
    (eq. p_costs); None is the quadratic cost, p_a = 2 on every axis."""
    if powers is None:
        return [2.0] * ndim
    pw = [float(q) for q in powers][:ndim]
    assert len(pw) == ndim and all(q > 1.0 for q in pw)
    return pw


def ctransform(f: np.ndarray, powers=None) -> np.ndarray:
    """f^c(x) = min_y c(x, y) - f(y) over all grid points y, with
    c(x, y) = 1/2|x - y|^2, or sum_a |x_a - y_a|^{p_a} / p_a (eq. p_costs).

    Separable decomposition (Section 4.1): start from u = -f and take the
    one-dimensional minimum along the last axis, then along each earlier axis;
    the iterated minimum equals the minimum over the whole grid."""
    u = -np.asarray(f, dtype=np.float64)
    pw = _powers(u.ndim, powers)
    for axis in reversed(range(u.ndim)):
        u = line_min(u, axis) if pw[axis] == 2.0 else line_min_p(u, axis, pw[axis])
    return u


def cost_matrix(shape: Sequence[int], powers=None) -> np.ndarray:
    """c(x_i, y_j) over all pairs of grid points (tiny grids only)."""
    pw = _powers(len(shape), powers)
    xs = np.stack([x.ravel() for x in np.meshgrid(*[(np.arange(n) + 0.5) / n for n in shape],
                                                    indexing="ij")], axis=1)
    d = np.abs(xs[:, None, :] - xs[None, :, :])
    return sum(d[..., a] ** pw[a] / pw[a] for a in range(len(shape)))


def ctransform_bruteforce(f: np.ndarray, powers=None) -> np.ndarray:
    """Non-separable O(N^2) version of the same definition (tiny grids only)."""
    c = cost_matrix(f.shape, powers)
    return (c - f.ravel()[None, :]).min(axis=1).reshape(f.shape)


# ---------------------------------------------------------------------------
# map T = x - grad f^c  and pushforward T#mu
# ---------------------------------------------------------------------------

def grad_fd(p: np.ndarray) -> List[np.ndarray]:
    """Central differences inside, one-sided differences on the two faces."""
    out = []
    for a, n in enumerate(p.shape):
        h = 1.0 / n
        g = np.empty_like(p)
        sl = lambda s: tuple(s if b == a else slice(None) for b in range(p.ndim))
        g[sl(slice(1, n - 1))] = (p[sl(slice(2, n))] - p[sl(slice(0, n - 2))]) / (2.0 * h)
        g[sl(slice(0, 1))] = (p[sl(slice(1, 2))] - p[sl(slice(0, 1))]) / h
        g[sl(slice(n - 1, n))] = (p[sl(slice(n - 1, n))] - p[sl(slice(n - 2, n - 1))]) / h
        out.append(g)
    return out


def transport_map(pc: np.ndarray, powers=None) -> List[np.ndarray]:
    """T(x) = x - (grad h)^{-1}(grad p^c(x)) (Lemma on c-transform properties
    (ii)), clamped to [h/2, 1 - h/2] per axis.  For the quadratic cost
    (grad h)^{-1} is the identity; for h_a(z) = |z|^p / p, h_a'(z) =
    sign(z)|z|^{p-1}, whose inverse is g -> sign(g)|g|^{1/(p-1)}."""
    xs = centres(pc.shape)
    pw = _powers(pc.ndim, powers)
    out = []
    for a, (x, g) in enumerate(zip(xs, grad_fd(pc))):
        h = 1.0 / pc.shape[a]
        disp = g if pw[a] == 2.0 else np.sign(g) * np.abs(g) ** (1.0 / (pw[a] - 1.0))
        out.append(np.clip(x - disp, 0.5 * h, 1.0 - 0.5 * h))
    return out


def pushforward(density: np.ndarray, T: Sequence[np.ndarray]) -> np.ndarray:
    """rho = T#density with piecewise-multilinear test functions: each cell's
    mass density*cell_volume is split over the 2^d cell centres around T(x)
    with the multilinear weights; returns a density (mass / cell_volume)."""
    shape = density.shape
    d = len(shape)
    m = (np.asarray(density, dtype=np.float64)).ravel()
    lo, w = [], []
    for a, n in enumerate(shape):
        t = np.asarray(T[a], dtype=np.float64).ravel() * n - 0.5
        i0 = np.minimum(np.floor(t), n - 2).astype(np.int64)
        i0 = np.maximum(i0, 0)
        lo.append(i0)
        w.append(t - i0)
    strides = [int(np.prod(shape[a + 1:])) for a in range(d)]
    rho = np.zeros(m.size, dtype=np.float64)
    for corner in range(1 << d):
        idx = np.zeros(m.size, dtype=np.int64)
        wt = np.ones(m.size, dtype=np.float64)
        for a in range(d):
            bit = (corner >> (d - 1 - a)) & 1
            idx += (lo[a] + bit) * strides[a]
            wt *= w[a] if bit else (1.0 - w[a])
        rho += np.bincount(idx, weights=m * wt, minlength=m.size)
    return rho.reshape(shape)


def displacement_interpolant(density: np.ndarray, pc: np.ndarray, t: float, powers=None) -> np.ndarray:
    """rho_t = S_t # density with S_t(x) = t T(x) + (1 - t) x, T the discrete
    map of pc (``transport_map``): the displacement interpolant between the
    two marginals of the transport (Section 4.3, optimal transport of
    images), deposited like the method's pushforward."""
    xs = centres(density.shape)
    T = transport_map(pc, powers)
    S = [t * Ta + (1.0 - t) * x for Ta, x in zip(T, xs)]
    return pushforward(density, S)


def primal_cost(density: np.ndarray, T: Sequence[np.ndarray], powers=None) -> float:
    """P = integral of c(x, T(x)) d(density): 1/2 |x - T(x)|^2, or
    sum_a |x_a - T_a(x)|^{p_a} / p_a."""
    xs = centres(density.shape)
    if powers is None:
        sq = sum((x - t) ** 2 for x, t in zip(xs, T))
        return cell_vol(density.shape) * float(np.sum(density * 0.5 * sq))
    pw = _powers(density.ndim, powers)
    c = sum(np.abs(x - t) ** q / q for x, t, q in zip(xs, T, pw))
    return cell_vol(density.shape) * float(np.sum(density * c))


# ---------------------------------------------------------------------------
# H^1 gradient: Neumann Poisson solve
# ---------------------------------------------------------------------------

def laplacian_eigenvalues(shape: Sequence[int]) -> np.ndarray:
    """lambda_k = sum_a (2 - 2 cos(pi k_a / n_a)) / h_a^2 for the
    second-difference Neumann Laplacian diagonalised by the DCT-II."""
    d = len(shape)
    lam = np.zeros(tuple(shape), dtype=np.float64)
    for a, n in enumerate(shape):
        k = np.arange(n, dtype=np.float64)
        s = [1] * d
        s[a] = n
        lam = lam + ((2.0 - 2.0 * np.cos(np.pi * k / n)) * n * n).reshape(s)
    return lam


def poisson_neumann(f: np.ndarray):
    """g = (-Laplacian)^{-1}(f - mean f), zero-flux Neumann, mean(g) = 0.

    Returns (g, G) with G = cell_volume * sum(f * g) = ||f - mean f||^2 in
    H^{-1} = ||grad g||^2_{L^2}, i.e. the squared H^1 norm of the gradient."""
    fh = scipy.fft.dctn(np.asarray(f, dtype=np.float64), type=2, norm="ortho", workers=WORKERS)
    lam = laplacian_eigenvalues(f.shape)
    lam.flat[0] = 1.0
    gh = fh / lam
    gh.flat[0] = 0.0
    G = cell_vol(f.shape) * float(np.sum(fh * gh))
    g = scipy.fft.idctn(gh, type=2, norm="ortho", workers=WORKERS)
    return g, G


# ---------------------------------------------------------------------------
# dual functional and step-size rule
# ---------------------------------------------------------------------------

def dual_value(p: np.ndarray, pc: np.ndarray, tgt: np.ndarray, src: np.ndarray) -> float:
    """J(p) = int p d(tgt) + int p^c d(src)  (eq. defJ; eq. defI with roles swapped)."""
    return cell_vol(p.shape) * (float(np.sum(p * tgt)) + float(np.sum(pc * src)))


@dataclass
class Params:
    max_iters: int = 60
    tol: float = 0.0
    sigma0: float = 0.0          # <= 0: 8 min(1/max mu, 1/max nu)
    sigma_min: float = 0.01
    beta1: float = 0.25
    beta2: float = 0.75
    alpha1: float = 1.25
    alpha2: float = 0.8
    powers: Optional[Tuple[float, ...]] = None   # eq. p_costs exponents per axis; None: quadratic


def initial_sigma(mu: np.ndarray, nu: np.ndarray) -> float:
    """Section 4.2: sigma = 8 min(||mu||_inf^{-1}, ||nu||_inf^{-1})."""
    return 8.0 * min(1.0 / float(np.max(mu)), 1.0 / float(np.max(nu)))


def update_sigma(sigma: float, increase: float, G: float, p: Params) -> float:
    """Section 4.2: keep sigma when beta1 sigma G <= increase <= beta2 sigma G;
    shrink by alpha2 (not below sigma_min) when the increase is too small, grow
    by alpha1 when it is too large."""
    if increase < p.beta1 * sigma * G:
        return max(p.alpha2 * sigma, p.sigma_min)
    if increase > p.beta2 * sigma * G:
        return p.alpha1 * sigma
    return sigma


# ---------------------------------------------------------------------------
# Algorithm 1
# ---------------------------------------------------------------------------

@dataclass
class Result:
    phi: np.ndarray
    psi: np.ndarray
    T: List[np.ndarray]
    dual: float
    primal: float
    gap: float
    G: float
    sigma: float
    iters: int
    converged: bool
    trace: List[Dict[str, float]] = field(default_factory=list)

    @property
    def w2sq(self) -> float:
        return 2.0 * self.dual


def half_step(p, src, tgt, sigma, prm: Params, pc=None):
    """One gradient step of the back-and-forth method on J(p) = <p,tgt> + <p^c,src>.

    phi-step: (p, src, tgt) = (phi, mu, nu); psi-step: (psi, nu, mu).
    Returns a dict with the head quantities (at p) and the stepped potential
    p + sigma grad J(p) together with its c-transform."""
    if pc is None:
        pc = ctransform(p, prm.powers)
    J0 = dual_value(p, pc, tgt, src)
    T = transport_map(pc, prm.powers)
    rho = pushforward(src, T)
    P = primal_cost(src, T, prm.powers)
    g, G = poisson_neumann(tgt - rho)
    return dict(pc=pc, J0=J0, T=T, rho=rho, P=P, g=g, G=G)


def solve(mu: np.ndarray, nu: np.ndarray, prm: Optional[Params] = None,
          phi_init: Optional[np.ndarray] = None) -> Result:
    """Back-and-forth iteration (Algorithm 1) with the Section 4.2 step rule.

    Iteration n: phi-step  phi_{n+1/2} = phi_n + sigma grad J(phi_n),
                           psi_{n+1/2} = (phi_{n+1/2})^c;
                 psi-step  psi_{n+1} = psi_{n+1/2} + sigma grad I(psi_{n+1/2}),
                           phi_{n+1} = (psi_{n+1})^c.
    sigma is one shared step, updated after each gradient step from the
    increase of the functional that step ascended.  The head of every
    iteration evaluates D_n = J(phi_n), the primal cost P_n of T_{phi_n} and
    G_n = ||nu - T#mu||^2_{H^-1}; gap_n = max(|P_n - D_n|, G_n).  The loop stops
    when gap_n < tol (tol > 0) or after max_iters iterations; the outputs are
    those of the last head evaluated (phi_final, its c-transform, its map)."""
    prm = prm or Params()
    mu = np.asarray(mu, dtype=np.float64)
    nu = np.asarray(nu, dtype=np.float64)
    phi = np.zeros_like(mu) if phi_init is None else np.array(phi_init, dtype=np.float64)
    sigma = prm.sigma0 if prm.sigma0 > 0 else initial_sigma(mu, nu)
    trace = []
    converged = False
    it = 0
    while True:
        head = half_step(phi, mu, nu, sigma, prm)
        gap = max(abs(head["P"] - head["J0"]), head["G"])
        trace.append(dict(iter=it, dual=head["J0"], primal=head["P"], G=head["G"],
                          gap=gap, sigma=sigma))
        if prm.tol > 0 and gap < prm.tol:
            converged = True
            break
        if it >= prm.max_iters:
            break
        # phi-step (Algorithm 1, first two lines)
        phi_half = phi + sigma * head["g"]
        psi = ctransform(phi_half, prm.powers)
        J1 = dual_value(phi_half, psi, nu, mu)
        trace[-1]["J_half"] = J1
        sigma = update_sigma(sigma, J1 - head["J0"], head["G"], prm)
        # psi-step (Algorithm 1, last two lines)
        hp = half_step(psi, nu, mu, sigma, prm)
        psi_new = psi + sigma * hp["g"]
        phi = ctransform(psi_new, prm.powers)
        I1 = dual_value(psi_new, phi, mu, nu)
        trace[-1].update(I_old=hp["J0"], I_new=I1, G_psi=hp["G"], sigma_psi=sigma)
        sigma = update_sigma(sigma, I1 - hp["J0"], hp["G"], prm)
        it += 1
    pc = head["pc"]
    m = float(np.mean(phi))
    return Result(phi=phi - m, psi=pc + m, T=head["T"], dual=head["J0"], primal=head["P"],
                  gap=gap, G=head["G"], sigma=sigma, iters=it, converged=converged, trace=trace)


def solve_ga(mu: np.ndarray, nu: np.ndarray, prm: Optional[Params] = None,
             phi_init: Optional[np.ndarray] = None) -> Result:
    """Plain H^1 gradient ascent on J, the scheme Section 4.3 compares the
    back-and-forth method with (Tables 5 and 6):

        phi_{n+1/2} = phi_n + sigma grad J(phi_n),   phi_{n+1} = (phi_{n+1/2})^cc.

    Only phi-space is visited.  The inner c-transform q = (phi_{n+1/2})^c is
    also phi_{n+1}^c, because f^ccc = f^c (Lemma on c-transform properties),
    so the head of iteration n+1 evaluates J(phi_{n+1}) with phi_{n+1}^c = q:
    two c-transforms and one Poisson solve per iteration, as the paper counts
    them.  sigma follows the Section 4.2 rule after each gradient step (the
    increase J(phi_{n+1/2}) - J(phi_n) against sigma G_n); the head, gap,
    stopping test and outputs are those of solve()."""
    prm = prm or Params()
    mu = np.asarray(mu, dtype=np.float64)
    nu = np.asarray(nu, dtype=np.float64)
    phi = np.zeros_like(mu) if phi_init is None else np.array(phi_init, dtype=np.float64)
    sigma = prm.sigma0 if prm.sigma0 > 0 else initial_sigma(mu, nu)
    pc = ctransform(phi, prm.powers)
    trace = []
    converged = False
    it = 0
    while True:
        head = half_step(phi, mu, nu, sigma, prm, pc=pc)
        gap = max(abs(head["P"] - head["J0"]), head["G"])
        trace.append(dict(iter=it, dual=head["J0"], primal=head["P"], G=head["G"],
                          gap=gap, sigma=sigma))
        if prm.tol > 0 and gap < prm.tol:
            converged = True
            break
        if it >= prm.max_iters:
            break
        phi_half = phi + sigma * head["g"]
        q = ctransform(phi_half, prm.powers)
        J1 = dual_value(phi_half, q, nu, mu)
        trace[-1]["J_half"] = J1
        sigma = update_sigma(sigma, J1 - head["J0"], head["G"], prm)
        phi = ctransform(q, prm.powers)
        pc = q
        it += 1
    m = float(np.mean(phi))
    return Result(phi=phi - m, psi=head["pc"] + m, T=head["T"], dual=head["J0"], primal=head["P"],
                  gap=gap, G=head["G"], sigma=sigma, iters=it, converged=converged, trace=trace)


def w2_gradients(res: Result, shape: Sequence[int]):
    """Envelope gradients of W2^2 = 2 C(mu, nu) w.r.t. the grid density values:
    d/dmu = 2 cell_volume (psi - mean psi), d/dnu = 2 cell_volume (phi - mean phi)
    (first variation of J, Lemma fact:derivative-J, at the maximiser)."""
    v = cell_vol(shape)
    return 2.0 * v * (res.psi - res.psi.mean()), 2.0 * v * (res.phi - res.phi.mean())
