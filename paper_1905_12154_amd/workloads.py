"""Seeded synthetic densities for the back-and-forth solver.

This module only draws and samples input densities; it holds none of the
method's arithmetic, so both the HIP path and the CPU oracle may consume its
output.  Every density is sampled at cell centres x = (i + 1/2) / n of a
uniform grid on [0, 1]^d (axis d-1 contiguous), in float64, and normalised so
that cell_volume * sum(density) = 1 (unit mass, mean value 1).

Workloads (shapes and value laws follow the paper's experiments, Section 4.3,
and the synthetic mixtures used for throughput measurement):

* ``gaussian_mixture``  - isotropic Gaussian bumps, equal weights.
* ``ellipses``          - union of uniform ellipses (zero density elsewhere).
* ``disks_ratio``       - indicator-of-disks density whose max/mean ratio is
                          pinned (default 50) by raising the smallest disk.
* ``two_discs`` / ``two_balls``            - Section 4.3, translation examples.
* ``square_to_four`` / ``cube_to_eight``   - Section 4.3, discontinuous maps.
* ``translated_pair``   - a density and its copy shifted by whole cells.

Seeds: numpy ``default_rng(SeedSequence([cfg, pair, side, which]))`` with
which = 0 for mu and 1 for nu.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Sequence, Tuple

import numpy as np

SIDES_C5 = (128, 256, 384, 512, 768, 1024)


def _rng(cfg: int, pair: int, side: int, which: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([cfg, pair, side, which]))


def cell_centres(shape: Sequence[int]) -> List[np.ndarray]:
    """Open-mesh cell-centre coordinates, one broadcastable array per axis."""
    d = len(shape)
    out = []
    for a, n in enumerate(shape):
        x = (np.arange(n, dtype=np.float64) + 0.5) / n
        s = [1] * d
        s[a] = n
        out.append(x.reshape(s))
    return out


def cell_volume(shape: Sequence[int]) -> float:
    return float(np.prod([1.0 / n for n in shape]))


def normalise(rho: np.ndarray) -> np.ndarray:
    rho = np.asarray(rho, dtype=np.float64)
    m = rho.sum() * cell_volume(rho.shape)
    if not (m > 0):
        raise ValueError("density has no mass")
    return rho / m


def gaussian_mixture(shape, centres, sigmas) -> np.ndarray:
    """Equal-weight mixture of isotropic Gaussians sampled at cell centres."""
    xs = cell_centres(shape)
    d = len(shape)
    rho = np.zeros(tuple(shape), dtype=np.float64)
    for c, s in zip(centres, sigmas):
        r2 = sum((xs[a] - c[a]) ** 2 for a in range(d))
        rho += np.exp(-r2 / (2.0 * s * s)) / (2.0 * math.pi * s * s) ** (d / 2.0)
    return normalise(rho)


def random_gaussian_mixture(shape, k, rng, lo=0.2, hi=0.8, smin=0.05, smax=0.15):
    d = len(shape)
    centres = rng.uniform(lo, hi, size=(k, d))
    sigmas = rng.uniform(smin, smax, size=k)
    return gaussian_mixture(shape, centres, sigmas)


def ellipses(shape, centres, semi_axes, angles) -> np.ndarray:
    """Union of uniform (value 1) ellipses in 2D, zero elsewhere."""
    assert len(shape) == 2
    x0, x1 = cell_centres(shape)
    inside = np.zeros(tuple(shape), dtype=bool)
    for c, (a, b), t in zip(centres, semi_axes, angles):
        dx0, dx1 = x0 - c[0], x1 - c[1]
        ct, st = math.cos(t), math.sin(t)
        u = ct * dx0 + st * dx1
        v = -st * dx0 + ct * dx1
        inside |= (u / a) ** 2 + (v / b) ** 2 <= 1.0
    return normalise(inside.astype(np.float64))


def _disks_raw(shape, centres, radii, heights):
    x0, x1 = cell_centres(shape)
    raw = np.zeros(tuple(shape), dtype=np.float64)
    for c, r, hgt in zip(centres, radii, heights):
        raw += hgt * (((x0 - c[0]) ** 2 + (x1 - c[1]) ** 2) <= r * r)
    return raw


def disks_ratio(shape, rng, ndisks=8, rmin=0.03, rmax=0.12, ratio=50.0, max_redraw=64):
    """Indicator-of-disks density with max/mean ratio pinned near ``ratio``.

    Radii U[rmin, rmax], centres U[r, 1-r]^2; all disks have height 1 except
    the smallest, whose height H is found by bisection so that
    max(rho)/mean(rho) = ratio (overlaps add).  Redraws when the target is out
    of reach (the smallest disk covers too much area)."""
    for _ in range(max_redraw):
        radii = rng.uniform(rmin, rmax, size=ndisks)
        centres = np.stack([rng.uniform(radii, 1.0 - radii), rng.uniform(radii, 1.0 - radii)], axis=1)
        s = int(np.argmin(radii))
        h_other = np.ones(ndisks)
        h_other[s] = 0.0
        base = _disks_raw(shape, centres, radii, h_other)
        h_small = np.zeros(ndisks)
        h_small[s] = 1.0
        mask = _disks_raw(shape, centres, radii, h_small) > 0
        if not mask.any():
            continue
        base_out = base[~mask].max() if (~mask).any() else 0.0
        base_in = base[mask].max()
        mean_base, frac = base.mean(), mask.mean()

        def raw_for(H):
            return base + H * mask

        def rat(H):
            return max(base_out, H + base_in) / (mean_base + H * frac)

        lo, hi = 1.0, 1.0e5
        if not (rat(lo) <= ratio <= rat(hi)):
            continue
        for _ in range(80):
            mid = math.sqrt(lo * hi)
            if rat(mid) < ratio:
                lo = mid
            else:
                hi = mid
        return normalise(raw_for(0.5 * (lo + hi)))
    raise RuntimeError("disks_ratio: could not reach the density ratio")


def two_discs(n: int):
    """Section 4.3: uniform discs of radius 1/8 centred at (1/4,1/4) and (3/4,3/4)."""
    x0, x1 = cell_centres((n, n))
    mu = ((x0 - 0.25) ** 2 + (x1 - 0.25) ** 2 <= 1.0 / 64).astype(np.float64)
    nu = ((x0 - 0.75) ** 2 + (x1 - 0.75) ** 2 <= 1.0 / 64).astype(np.float64)
    return normalise(mu), normalise(nu)


def crossing_discs(n: int):
    """Section 4.3, optimal transport with general costs: mu is two uniform
    discs of radius 1/8 centred at (1/4,1/4) and (3/4,3/4), nu two centred at
    (1/4,3/4) and (3/4,1/4)."""
    x0, x1 = cell_centres((n, n))
    r2 = 1.0 / 64
    disc = lambda c0, c1: (x0 - c0) ** 2 + (x1 - c1) ** 2 <= r2
    mu = (disc(0.25, 0.25) | disc(0.75, 0.75)).astype(np.float64)
    nu = (disc(0.25, 0.75) | disc(0.75, 0.25)).astype(np.float64)
    return normalise(mu), normalise(nu)


def two_balls(n: int):
    """Section 4.3: uniform balls of radius 1/8 centred at (1/4,..) and (3/4,..)."""
    x = cell_centres((n, n, n))
    mu = (sum((xa - 0.25) ** 2 for xa in x) <= 1.0 / 64).astype(np.float64)
    nu = (sum((xa - 0.75) ** 2 for xa in x) <= 1.0 / 64).astype(np.float64)
    return normalise(mu), normalise(nu)


def _box(x, lo, hi):
    m = np.ones(np.broadcast_shapes(*[xa.shape for xa in x]), dtype=bool)
    for xa, l, h in zip(x, lo, hi):
        m &= (xa >= l) & (xa <= h)
    return m


def square_to_four(n: int):
    """Section 4.3: square of side 1/4 centred at (1/2,1/2) to four squares of
    side 1/8 centred at (3/16 + 5i/8, 3/16 + 5j/8)."""
    x = cell_centres((n, n))
    mu = _box(x, (0.375, 0.375), (0.625, 0.625)).astype(np.float64)
    nu = np.zeros((n, n))
    for i in (0, 1):
        for j in (0, 1):
            c = (3 / 16 + 5 * i / 8, 3 / 16 + 5 * j / 8)
            nu += _box(x, (c[0] - 1 / 16, c[1] - 1 / 16), (c[0] + 1 / 16, c[1] + 1 / 16))
    return normalise(mu), normalise(nu)


def cube_to_eight(n: int):
    """Section 4.3: cube of side 1/4 centred at (1/2,1/2,1/2) to eight cubes of side 1/8."""
    x = cell_centres((n, n, n))
    mu = _box(x, (0.375,) * 3, (0.625,) * 3).astype(np.float64)
    nu = np.zeros((n, n, n))
    for i in (0, 1):
        for j in (0, 1):
            for k in (0, 1):
                c = [3 / 16 + 5 * t / 8 for t in (i, j, k)]
                nu += _box(x, [cc - 1 / 16 for cc in c], [cc + 1 / 16 for cc in c])
    return normalise(mu), normalise(nu)


def translated_pair(shape, shift_cells, rng, k=2, rmin=0.06, rmax=0.1):
    """mu = union of k uniform balls, nu = mu shifted by whole cells.

    The balls are placed so that the shifted copy stays inside the box, so nu
    is exactly mu(x - a) on the grid with a = shift_cells * h."""
    d = len(shape)
    xs = cell_centres(shape)
    mu = np.zeros(tuple(shape), dtype=np.float64)
    for _ in range(k):
        r = rng.uniform(rmin, rmax)
        c = [rng.uniform(r + 0.02 + max(0, -s) / n, 1 - r - 0.02 - max(0, s) / n)
             for s, n in zip(shift_cells, shape)]
        mu += (sum((xs[a] - c[a]) ** 2 for a in range(d)) <= r * r)
    mu = normalise(mu)
    nu = np.zeros_like(mu)
    src = tuple(slice(max(0, -s), n - max(0, s)) for s, n in zip(shift_cells, shape))
    dst = tuple(slice(max(0, s), n - max(0, -s)) for s, n in zip(shift_cells, shape))
    nu[dst] = mu[src]
    return mu, normalise(nu)


# ---------------------------------------------------------------------------
# The named synthetic configurations.
# ---------------------------------------------------------------------------

def config_c1():
    """64^2, mu and nu each a mixture of 3 isotropic Gaussians."""
    shape = (64, 64)
    mu = random_gaussian_mixture(shape, 3, _rng(1, 0, 64, 0))
    nu = random_gaussian_mixture(shape, 3, _rng(1, 0, 64, 1))
    return mu, nu


def config_c2(n: int = 1024):
    """n^2: mu = union of 5 uniform ellipses, nu = 4-Gaussian mixture."""
    shape = (n, n)
    r = _rng(2, 0, n, 0)
    centres = r.uniform(0.2, 0.8, size=(5, 2))
    axes = r.uniform(0.04, 0.15, size=(5, 2))
    angles = r.uniform(0.0, math.pi, size=5)
    mu = ellipses(shape, centres, axes, angles)
    nu = random_gaussian_mixture(shape, 4, _rng(2, 0, n, 1))
    return mu, nu


def config_c3(n: int = 4096):
    """n^2: 8-disk indicator densities with max/mean density ratio 50."""
    shape = (n, n)
    mu = disks_ratio(shape, _rng(3, 0, n, 0))
    nu = disks_ratio(shape, _rng(3, 0, n, 1))
    return mu, nu


def config_c4(n: int = 384):
    """n^3: 6-Gaussian mixtures, sigma U[0.04, 0.12]."""
    shape = (n, n, n)
    mu = random_gaussian_mixture(shape, 6, _rng(4, 0, n, 0), smin=0.04, smax=0.12)
    nu = random_gaussian_mixture(shape, 6, _rng(4, 0, n, 1), smin=0.04, smax=0.12)
    return mu, nu


def c5_sides(npairs: int = 64, sides: Sequence[int] = SIDES_C5) -> List[int]:
    r = np.random.default_rng(np.random.SeedSequence([5, 0xC5]))
    return [int(s) for s in r.choice(np.asarray(sides), size=npairs)]


def config_c5_pair(pair: int, side: int):
    """One pair of the batched workload: 2-6 component mixtures of C1's law."""
    shape = (side, side)
    out = []
    for which in (0, 1):
        r = _rng(5, pair, side, which)
        k = int(r.integers(2, 7))
        out.append(random_gaussian_mixture(shape, k, r))
    return out[0], out[1]


def config_c5(npairs: int = 64, sides: Sequence[int] = SIDES_C5):
    return [config_c5_pair(p, s) for p, s in enumerate(c5_sides(npairs, sides))]


@dataclass
class Workload:
    name: str
    mu: np.ndarray
    nu: np.ndarray
    meta: dict = field(default_factory=dict)


def load(name: str, **kw) -> Workload:
    table = {
        "c1": config_c1, "c2": config_c2, "c3": config_c3, "c4": config_c4,
    }
    mu, nu = table[name](**kw)
    return Workload(name, mu, nu, dict(kw))
