"""MI355X (gfx950) solver-free componentwise ADMM for multi-phase linearised
distribution OPF.

The compute path is the HIP library `libopf_admm.so` behind the C ABI of
include/opf_admm.h; `binding` marshals arguments to it.  There is no CPU
fallback: using the solver without the built library raises."""
from . import binding
from .binding import (OPF_ADMIT_ARRIVAL, OPF_ADMIT_LARGEST_FIRST, OPF_KERNEL_AUTO, OPF_KERNEL_PERSISTENT,
                      OPF_KERNEL_STEP, OPF_KERNEL_TILED, OPF_PREC_FP64,
                      OPF_PREC_MIXED, OPF_RHO_LAG, OPF_RHO_PLAIN, OPF_RHO_RELATIVE, BatchSolver, OpfError, Server,
                      Solver)

__all__ = ["binding", "Solver", "BatchSolver", "Server", "OpfError", "OPF_PREC_FP64", "OPF_PREC_MIXED", "OPF_KERNEL_AUTO",
           "OPF_KERNEL_STEP", "OPF_KERNEL_PERSISTENT", "OPF_KERNEL_TILED", "OPF_RHO_RELATIVE", "OPF_RHO_PLAIN",
           "OPF_RHO_LAG", "OPF_ADMIT_LARGEST_FIRST", "OPF_ADMIT_ARRIVAL"]
