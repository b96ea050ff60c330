"""Plain FP64 CPU oracle for SPOCK (Chambolle-Pock + SuperMann/Anderson on the
risk-averse splitting of arXiv 2212.01110).

TEST INFRASTRUCTURE ONLY. Nothing in the product package may import, call or
link this package; only the tests, the smoke check and the CPU-baseline leg of
the benchmark do. It shares no code with the GPU path: the only common
dependency is the seeded input generator `spock_gen`, which holds no solver
arithmetic.

Modules, each citing the passage it follows:
  layout     canonical ordering of z and eta (section 5.2, operator splitting)
  operators  L, L* and ||L|| (section 5.2 and the block-diagonal remark after it)
  prox       Alg. 1, Alg. 2, the S2 kernel projection, prox of g* (sections 5.3, 5.4)
  cp         the CP operator T, residual, xi, omega, vanilla CP (section 3)
  spock      Anderson directions and SPOCK (section 6, Alg. 3)
  risk       AV@R and the exact nested cost of a policy (section 4.2, eq. original-problem)
  sensitivity envelope gradients of V*, and implicit (fixed-point) tangents of V* and
              u^0 w.r.t. x0 and the cost weights (section 3)

Pins (tests/test_oracle_*.py) tie every function to the mathematics rather
than to itself: L/L* by the adjoint identity and a feasible conic point built
from the AV@R dual; ||L|| by the full spectral norm and power iteration; S1 by
dense affine projection; S2 by a null-space basis; prox g* by its optimality
conditions; T by firm nonexpansiveness and the certificates of section 3; the
whole solver by the risk-neutral tree-LQR closed form and by brute-force
nested dynamic programming.
"""
from .layout import Layout
from .operators import L_apply, Lt_apply, norm_L, dense_L
from .prox import (factor_s1, proj_S1, proj_S2_block, proj_S2, prox_f,
                   proj_S3, prox_gstar, proj_soc)
from .cp import (Problem, T_apply, residual_stats, M_apply, cp_solve, Settings,
                 SolveResult)
from .spock import spock_solve, AndersonBuffer
from .risk import avar, nested_cost
from .sensitivity import envelope_gradients, fixed_point_tangent, implicit_gradients, T_jvp

__all__ = [
    "Layout", "L_apply", "Lt_apply", "norm_L", "dense_L", "factor_s1", "proj_S1",
    "proj_S2_block", "proj_S2", "prox_f", "proj_S3", "prox_gstar", "proj_soc",
    "Problem", "T_apply", "residual_stats", "M_apply", "cp_solve", "Settings", "SolveResult",
    "spock_solve", "AndersonBuffer", "avar", "nested_cost", "envelope_gradients",
    "fixed_point_tangent", "implicit_gradients", "T_jvp",
]
