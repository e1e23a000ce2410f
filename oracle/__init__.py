"""Plain float64 CPU oracle of MIS-SLAM's deformable registration hot path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke entry point and the
benchmark's CPU-baseline leg may import this package.  The GPU library never
calls it and shares no code with it.

Each function follows one passage of the paper (arXiv:1803.02009), cited by
section and equation number as numbered in the LaTeX source order:
  Eq.(1) ED warp (Sec. II-D)          Eq.(2) skinning weight (Sec. II-D)
  Eq.(3) total energy (Sec. II-E)     Eqs.(4)-(5) rotation term
  Eq.(6) regularisation term          Eq.(7) visibility gates
  Eq.(8) point-to-plane data term     Eq.(9) key-point correspondence term  Eq.(10) global pose terms (joint pose + ED)
  Sec. II-F optimisation (LM: damped GN + PCG, fixed or adaptive damping)
  Alg. 1/2 registration and fusion    Eqs.(12)-(15) fusion update (Sec. II-G)
  Alg. 2 steps 3-5, Alg. 3            growth, removal, down-sampling, node regeneration
Where the paper is silent or garbled the reading taken is stated in the
function's docstring.  Everything is float64 numpy; inputs arrive as float32
values promoted exactly.

Parameter layout: x_j = (c1, c2, c3, t_j) in R^12, where A_j = [c1 c2 c3]
column by column (the c's of Eq.(5)); x[3c + a] = A_j[a, c], x[9 + a] = t_j[a].
"""
from .graph import knn, skin_weights, node_graph, bsr_pattern, build_graph  # noqa: F401
from .warp import ed_warp, warp_normals, identity_params  # noqa: F401
from .depthmap import vertex_map, normal_map  # noqa: F401
from .assoc import associate  # noqa: F401
from .energy import rot_residuals, reg_residuals, energies  # noqa: F401
from .system import (data_jacobian_rows, rot_jacobian, reg_jacobian, dense_system,  # noqa: F401
                     block_system, dense_from_blocks)
from .pcg import block_jacobi, pcg, cholesky_solve  # noqa: F401
from .gn import gn_register, Problem  # noqa: F401
from .grad import energy_grad_params, energy_grad_points, total_energy_fixed  # noqa: F401
from .fuse import fuse, fuse_warped, zbuffer  # noqa: F401
from .mixed import round_bf16, round_fp16  # noqa: F401
from .grow import grow, voxel_keys  # noqa: F401
from .corr import corr_residuals, corr_jacobian_rows, corr_energy  # noqa: F401
from .lm import LMSchedule, lm_iterate, lm_register, objective  # noqa: F401
from .pose import joint_register, joint_linearize, joint_pcg, so3_exp, so3_log  # noqa: F401
