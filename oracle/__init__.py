"""FP64 CPU oracle for the maximal-entropy moment method (MEM) hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, links or
executes this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may use it.  It shares no code, tables or
constants with the HIP library in ``paper_2303_02898_amd``; the only module both
sides read is ``mem_inputs`` (seeded workload generators).

The oracle is deliberately plain: NumPy in float64, batched over cells with
masks, direct weighted sums over quadrature nodes (no basis-product table), and
the algorithm steps in the paper's order.  Module map (paper sections):

* ``quadrature`` -- the numerical integration rule (Sec. 3.1, eq. "Numerical
  integration"), here tensor Gauss--Hermite in gauge coordinates.
* ``basis``      -- sufficient statistics: orthonormal Hermite products up to
  total degree 4 (App. B, the orthogonal form of the 35-moment system).
* ``maxent``     -- canonical form, log-sum-exp partition function (Sec. 3.1),
  dual objective, gradient and Hessian (App. C), modified Newton with the
  Armijo backtracking line search (Alg. 1).
* ``gauge``      -- Hermite gauge parameters (Sec. 3.3) and change of gauge
  T(g', g) (eq. "Change gauge M F"), built by numerical projection.
* ``flux``       -- moment fluxes (eq. "The ME equation", flux line) and the
  characteristic speeds used by local Lax--Friedrichs (Sec. 3.4).
* ``kinetics``   -- ES-BGK collision (App. A), normal-shock set-up (App. D),
  LLF finite volume in local gauges and the time step of Alg. 2.
* ``workloads``  -- oracle-side construction of targets that need the
  parameter-to-moment map (the 1D perturbed-multiplier workload).
* ``axisym``     -- the paper's own discretisation: nine statistics of
  (u_x, u_r), block-wise Gauss--Legendre on a truncated box fixed in physical
  velocity, the integration-domain formula, per-cell Phi in the gauge, moments,
  fluxes, Hermite gauge and Alg. 1 on it.

Pins: every function here is checked in ``tests/test_oracle_*.py`` against
closed forms, invariants or brute force (never against itself or the GPU).
"""

from . import quadrature, basis, maxent, gauge, flux, kinetics, axisym  # noqa: F401
