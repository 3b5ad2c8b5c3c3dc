"""Plain FP64 CPU oracle for the spectral complex-valued Stokes method.

TEST INFRASTRUCTURE ONLY. Nothing on the product path may import this
package: only the tests, the smoke check and the benchmark's CPU-baseline leg
use it. It shares no code with the HIP library and is written for
readability, not speed.

What it computes (the paper's section 2):
* quadratic-velocity / linear-pressure (Taylor-Hood) numbering and sparsity
  (section 2.3, Eq. shape_fun);
* element integrals of the stiffness, mass and gradient-coupling matrices by
  direct quadrature in physical space (section 2.3, Eq. LS_construction);
* boundary traction loads and Dirichlet data (Eqs. dir_dis, LS_construction);
* for every Fourier mode the complex saddle-point system, solved by a sparse
  direct LU factorization (section 2.4, step 3);
* the time reconstruction of the modes (section 2.4, step 4);
* closed-form channel and pipe solutions (section 3.2, 3.4) for pinning.

Parity status: every function is pinned by tests under tests/test_oracle_*.py
except where a docstring says "parity unpinned".
"""
from .quadrature import gm_rule  # noqa: F401
from .numbering import p2_numbering, s2_pattern, c21_pattern  # noqa: F401
from .assemble import assemble, boundary_loads, bc_nodes  # noqa: F401
from .solve import system_matrix, system_rhs, solve_modes, solve_case  # noqa: F401
from .synth import synthesize  # noqa: F401
from . import exact  # noqa: F401
