"""FP64 CPU oracle for the WaveHoltz-filter eigensolver (EigenWave).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the tests, the smoke check and the CPU-baseline leg
of the benchmark do.  It shares no code with the HIP library (it imports only
numpy/scipy and the seeded input generators in ``synthetic``).

Every routine is a plain, slow restatement of the paper's definitions in
double precision, written so that it can be checked against the paper by eye:

* ``discrete``  -- grids, the order-2/4 Dirichlet Laplacian L_h, its closed-form
  eigenpairs, the continuous and discrete filter functions, alpha_d, the
  adjusted frequency and the time-step plan (Sec. "Discrete approximations",
  "Discrete time-stepping analysis").
* ``wave``      -- one wave-solve plus trapezoidal time filter, S v, with
  explicit leapfrog or implicit trapezoidal stepping (eqs. explicitScheme,
  implicitScheme, filterQuadrature).
* ``mg``        -- plain geometric multigrid for M = I - (dt^2/2) L_h.
* ``eigs``      -- Arnoldi with modified Gram-Schmidt (Alg. "Arnoldi"),
  Krylov-Schur restarting, and the Rayleigh quotient stage.
* ``cnn``       -- the small convolutional warm-start network, forward and
  backward, in FP64.
* ``walls``     -- boxes with Neumann walls: the Laplacian with even-reflection
  ghosts, its closed-form eigenpairs and symmetrising weights, and the
  explicit wave-solve.
* ``mapped``    -- a single curvilinear grid (mapping method): the order-2
  conservative Laplacian with metric terms of the grid coordinates, its
  J-weighted symmetry, Gershgorin time plan and explicit wave-solve.

Readings of the paper where it is silent (boundary closure for order 4,
trapezoid weights, CFL definition, ...) are stated in each function.
Parity status: every function here is pinned by a ``-m "not gpu"`` test in
``tests/test_oracle_*.py`` against closed forms, printed paper values, dense
eigensolves or brute force; none is "parity unpinned".
"""
