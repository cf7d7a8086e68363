"""MI355X space-time FMM for the heat equation (single- and double-layer apply,
Dirichlet solve).

The compute path lives in the HIP library ``libpfmm.so`` (see include/pfmm.h);
this package only loads it and marshals arguments.
"""
from .pfmm import (PfmmError, Params, SolveOpts, SolveInfo, Tree, Batch, Precond, default_params, plan_stats, lib_path,
                   load_library, STATUS_NAMES, PROFILE_STAGES, FP64, MIXED_FP32, MIXED_BF16, NF_STORED,
                   NF_TOEPLITZ, OP_V, OP_K, OP_K1)

__all__ = ["PfmmError", "Params", "SolveOpts", "SolveInfo", "Tree", "Batch", "Precond", "default_params", "plan_stats", "lib_path",
           "load_library", "STATUS_NAMES", "PROFILE_STAGES", "FP64", "MIXED_FP32", "MIXED_BF16", "NF_STORED",
           "NF_TOEPLITZ", "OP_V", "OP_K", "OP_K1"]
