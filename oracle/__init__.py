"""Plain FP64 CPU oracle for Gauss-Newton accelerated MPPI (arXiv 2512.04579).

TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test suite, the smoke check of
the graft entry point and the ``cpu_baseline`` leg of the benchmark may import
or run anything in this package.  The GPU library never calls into it, and it
shares no code, tables or constants with the GPU path: inputs come from the
``workloads`` module (seeded data only) and every piece of arithmetic here is
written out from the paper in NumPy float64.

Contents and what follows which passage:

* ``dynamics``  -- the black-box simulator F of Eq. (1) for the double
  integrator of Problem IV and the RK4-discretised spring chain (RK4 as in
  Problem V, Sec. 5).
* ``ocp``       -- single-shooting rollouts, the least-squares residual R and
  the cost C = Phi(R) = 1/2 ||R||^2 of Eqs. (2) and (4).
* ``mppi``      -- sample weights and the weighted-mean MPPI step,
  Eqs. (5)-(8).
* ``jacobian``  -- Gaussian-smoothing Jacobian reconstruction, Eq. (10), in
  its Monte-Carlo form and in the least-squares form; central finite
  differences (Method A, Sec. 5) as a reference.
* ``ggn``       -- the GGN step of Eq. (13) and the line search of
  Eqs. (14)-(15).
* ``solvers``   -- Alg. 1 (GN-MPPI, Methods D/E), plain MPPI (Method C) and
  GGN with finite differences (Method A).
* ``lqr``       -- finite-horizon Riccati recursion and the dense QP of the
  linear-quadratic Problem IV: the exact optimum GN-MPPI must hit.
* ``philox``    -- Philox4x32-10 (Salmon et al., SC'11) and Box-Muller, to
  check the device sampler element by element.
* ``sigma_points`` -- the deterministic Dirac-mixture perturbation set of
  Method E (Sec. 5).

Every function has at least one pin in ``tests/test_oracle_*.py`` that does
not reuse its own formula (closed forms, brute force, invariants, a second
route).  The only result without such a pin is the end-to-end trajectory of
Alg. 1 on the nonlinear chain: parity unpinned beyond the per-step pins.
"""

from . import dynamics, ocp, mppi, jacobian, ggn, solvers, lqr, philox, sigma_points  # noqa: F401
