"""CPU float64 oracle of the back-and-forth method -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import, call, link or execute anything in this package.  It
shares no code with the HIP path (``paper_1905_12154_amd``) and neither imports
the other; both consume the seeded densities of
``paper_1905_12154_amd.workloads``, which hold none of the method's arithmetic.

Pins (see tests/test_oracle_*.py):
  * ctransform       -- non-separable brute force of the definition, c-transform
                        identities (Lemma on c-transform properties, (i)),
                        closed form for linear potentials.
  * poisson_neumann  -- residual of the second-difference stencil applied
                        directly, sparse direct solve, summation-by-parts for G.
  * pushforward      -- mass conservation, identity map, whole-cell shifts,
                        adjointness with multilinear interpolation (scipy).
  * update_sigma     -- scripted sequences against the Section 4.2 rule.
  * solve            -- exact costs of the Section 4.3 examples (discs 1/4,
                        squares 1/16, translations |a|^2/2), weak duality
                        against the exact discrete LP (HiGHS) on tiny grids,
                        the unconditional c-transform half of the monotone
                        chain, Gaussian-to-Gaussian affine maps.
  * solve_ga         -- iterates c-concave and psi = phi^c by the brute-force
                        transform (f^ccc = f^c), the double transform never
                        lowers J, weak duality against the LP and
                        feasibility, the exact two-disc cost, the first step
                        equal to the phi-step of Algorithm 1, and the
                        iteration ratio of Tables 5 and 6 (the
                        back-and-forth iteration needs several times fewer).
  * power costs      -- (eq. p_costs, powers=...) the separable transform
                        against the non-separable definition, p = 2 equal to
                        the quadratic line minimum, c-transform identities, the
                        map of a linear potential (a translation inverting
                        h'), the primal cost of a translation, exact costs of
                        translations (Jensen), weak duality against the LP,
                        and the crossing discs moving along one axis only at
                        cost 1/24 for exponents (3, 1.1).
  * displacement_interpolant -- t = 0 gives the density itself, t = 1 the
                        method's pushforward, whole-cell translations move by
                        t times the shift, mass is conserved, and the
                        interpolant of two Gaussians is the Gaussian with
                        interpolated mean and standard deviation.
  * w2_gradients     -- parity unpinned beyond finite differences of the
                        oracle's own value (the discretised pushforward adds an
                        envelope error of the order of the discretisation).
"""
from . import bfm  # noqa: F401
