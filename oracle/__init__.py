"""Plain CPU oracle for the DeepONet meta-solver hot path (complex128 numpy).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or
links this package: only the tests, the smoke check and the benchmark's
CPU-baseline leg use it.  It shares no code with the HIP library; the two
meet only at the seeded input arrays.

Every function states the passage of the paper it follows (section,
equation, appendix).  Where the paper is silent or garbled the reading taken
is stated in the function's docstring.

Modules
-------
operator   the discrete Helmholtz operator, its dense assembly, residual,
           damped Jacobi and red-black Gauss-Seidel sweeps   (§2 eq. 1, §3.1.1 eq. 2)
krylov     restarted GMRES(m) with CGS2 and BiCGStab, right-preconditioned  (§3.1.2)
deeponet   MLP branch/trunk networks and the DeepONet output head         (App. B)
coarse     trunk-basis prolongation, QR, Galerkin coarse matrix, M2     (App. C)
meta       relaxation meta-solver (eq. 3) and the Krylov preconditioner (§3.1.2, App. C)
adjoint    receiver misfit and its k^2 gradient by the conjugate-transpose solve  (§2 eq. 1)
training   DeepONet training step: relative L2 loss, backpropagation, Adam       (App. B)
multigrid  geometric V-cycle preconditioner with the DeepONet-Jacobi smoother  (§4.3)
"""
from . import operator, krylov, deeponet, coarse, meta, adjoint, training, multigrid  # noqa: F401
