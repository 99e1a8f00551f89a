"""FP64 CPU oracle for the hybrid FE/FD Maxwell forward / adjoint / gradient.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package may import, call or
execute this package; only the tests, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
path: it builds its own mesh, its own operators and its own time loop, plainly
and slowly, in float64 with numpy/scipy.

What it computes (the discrete scheme the GPU path must reproduce):

* Forward problem (paper, box "Forward problem", eq. forward_prob, and the
  model problem eq. model1 with the plane-wave source eq. f): explicit
  central-difference leapfrog of
      M_eps (E^{n+1} - 2E^n + E^{n-1})/dt^2 + (M_sigma + S^n)(E^{n+1} - E^{n-1})/(2 dt)
      + A E^n = F^n,
  with A = stiffness (7-point on the finite-difference rows, assembled P1 on
  the Kuhn tetrahedra of the FEM rows) plus the stabilising div-div term
  int div(lambda) div((eps - 1) E) of the weak form (eq. lagrangian_weak).
* Adjoint problem (box "Adjoint problem", eq. adjoint_prob): the exact
  transpose of that recursion, run backward from lambda^{N_t} = 0 with the
  trace misfit as source.
* Gradient (eq. gradeps and the optimality conditions dL/deps, dL/dsigma):
  the exact derivative of the discrete loss 1/2 sum |E - E_obs|^2 over
  detectors and steps with respect to nodal eps and sigma.
* General initial data (eq. forward_initial_cond): the starting levels E^0 = f_0,
  E^{-1} = f_0 - dt f_1 (start from rest by default), with the level-0 rows of the
  gradient that carry the -lambda(x, 0) f_1 term of eq. gradeps.
* Variants: the paper's own gradient formula, and the symmetric div-div form R2 for
  which that formula is the exact gradient (oracle/discretization.py).
* Reconstruction (box "CGA", oracle/cga.py): the conjugate gradient iteration on
  eps and sigma with the Tikhonov terms of eq. tikhonov_functional, the step-size
  and regularisation rules of the box and the coefficient box of
  eq. epsilon_sigma_constraint.

Parity pins live in ``tests/test_oracle_*.py``.  Parity unpinned: whether this
discretisation is the one of the paper's companion reference (the paper defers
the discretisation to it and prints no discrete values).
"""

from .discretization import Discretization  # noqa: F401
from .solver import (  # noqa: F401
    source_time_function, forward, adjoint_gradient, loss_and_cotangent, energy_balance_residual, taper,
)
