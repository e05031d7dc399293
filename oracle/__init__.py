"""CPU FP64 oracle for the fully implicit Runge-Kutta stage solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code, headers,
tables or helpers with the HIP library; it never reads a value produced by
the HIP path.

What it computes is the plain definition of one Runge-Kutta step of
``M u' = N(u, t)`` (paper, Section 1.1, equations (update) and (stages)),
and of its index-1 DAE form (Section 6, equation (dae_stage)):

* ``tableau``  -- Gauss and Radau IIA collocation tableaux, built in
  extended precision from the nodes' defining polynomials, plus the
  quantities of Sections 3-4 that the paper prints (eigenvalues of A0^{-1},
  gamma_*, the condition bound of Corollary 1, the d-weights of
  equation (Q0approx)).
* ``problems`` -- the semi-discrete operators N_h and their exact Jacobians
  (1-D viscous Burgers, 2-D nonlinear diffusion, 2-D vorticity-streamfunction
  with the Arakawa Jacobian), written with NumPy / SciPy sparse.
* ``newton``   -- the stage equations solved by full Newton with a direct
  sparse LU (SciPy SuperLU), iterated to stagnation, then the update.

Everything is float64 NumPy; pure-Python loops appear only in the
extended-precision tableau construction.
"""
