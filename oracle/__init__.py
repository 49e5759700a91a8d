"""CPU FP64 oracle for the explicit divergence-free DG scheme (test infrastructure).

This package is the plain, slow, obviously correct reference the GPU library is
checked against.  Only the test suite, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it; the product path never does.
It shares no code with the GPU library: its own quadrature, its own facet
matching, its own (global, conforming) BDM_k basis, its own residual and a sparse
direct solve of the global mixed system.

What it computes, in the paper's terms (G. Fu, "An explicit divergence-free DG
method for incompressible flow"):

* spaces: the H(div)-conforming BDM_k velocity space and the broken, mean-zero
  P^{k-1} pressure space (Sec. 2.1, eq. (space));
* the DG operator L(u)(v) = -C_h(u; u, v) - B_h(u, v): upwind convection
  (Sec. 2.2, eq. (adv)) and symmetric interior penalty viscosity with
  penalty alpha k^2 / h (Sec. 3, eq. (viscous));
* the divergence-free mass inversion as the global mixed Poisson problem
  (Sec. 2.4, eq. (FE2); Theorem 1), factored once with SuperLU;
* TVD-RK3 in mass-matrix form (Sec. 2.3, eq. (rk3));
* the hybrid-mixed system (eq. (FE3)) written out densely for tiny meshes, as a
  check of Theorem 2;
* diagnostics (energy, enstrophy, divergence, normal jumps) and a reverse-mode
  gradient of the final kinetic energy.

Parity pins live in ``tests/test_oracle_*.py``.  The functions whose only check
is agreement with another oracle function are marked "parity unpinned" in their
docstrings.
"""
from .quadrature import gauss_legendre_01, triangle_rule, facet_rule_points  # noqa: F401
from .mesh import OracleMesh  # noqa: F401
from .bdm import BDMSpace  # noqa: F401
from .scheme import Oracle  # noqa: F401
