"""MI355X (gfx950) Newton step of the VMS / generalized-alpha P1-tetrahedral
hyper-elastodynamics method with nested block-preconditioned FGMRES.

``libvms.so`` (HIP, built in-tree by ``python -m paper_1809_06350_amd.build``)
holds every step of the path; ``vms.Problem`` marshals torch tensors into its
C ABI (include/vms.h).
"""
from .vms import (Problem, Matrix, VmsError, solver_opts, newton_opts, time_int,  # noqa: F401
                  ASM_RESIDUAL, ASM_TANGENT, ASM_RKCORR, OP_FULL, OP_A, OP_B, OP_C, OP_D,
                  PC_LDU, PC_UPPER, PC_LOWER, PC_DIAG, FP64, MIXED, ORTH_CGS2, ORTH_MGS)
