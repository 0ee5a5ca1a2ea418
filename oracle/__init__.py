"""CPU oracle for MGRIT applied to method-of-lines discretizations of periodic
linear advection (De Sterck, Falgout, Krzysik, Schroder, arXiv 2209.06916).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and its
Python binding) may import, call or execute anything in this package; only the
test-suite, the smoke check in ``__graft_entry__`` and the ``cpu_baseline`` leg
of ``bench.py`` use it.  It shares no code with the GPU path: it has its own
stencils, tableaux, correction coefficients and (FFT-based) periodic solves.

Everything is plain numpy in float64, written from the paper's definitions:

* ``discretization`` -- upwind stencils L_p (Sec. 4.1), Runge-Kutta tableaux and
  stability functions (Sec. 4.2), the method-of-lines step (eq. MOL_M_def), the
  semi-Lagrangian step S_p (Sec. 3), the difference matrix D^(p+1) (eq. Dp+1_def),
  the correction coefficient phi (eqs. varphi-constant-MOL-SL and
  MOL-SL-corrected-multilevel) and the corrected coarse operator Psi
  (eq. MOL-SL-corrected).
* ``mgrit`` -- sequential time-stepping (eq. one-step-general) and linear
  two-level / multilevel MGRIT with F(CF)^nu relaxation (Sec. 2.2).
* ``lfa`` -- Fourier symbols and the two-level convergence estimate
  (eqs. rho-omega-theta, rho-asym) and the lower bound of Theorem 1
  (eq. rho-check-MOL).

Parity status of each function is stated in its docstring; every function is
pinned by a ``-m "not gpu"`` test against values the paper prints, closed forms,
exact special cases, brute force or convergence orders.  The one exception is
the fifth-order explicit tableau (see ``discretization.erk_tableau``), whose
stability polynomial the paper's two tables do not determine consistently:
parity unpinned for ERK5 against Table 2.
"""
