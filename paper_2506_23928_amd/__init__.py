"""MI355X (gfx950) implementation of trajectory-unravelled time-dependent variational Monte
Carlo (otVMC): a C-ABI library of HIP kernels (``libtvmc.so``) and its Python binding."""
from .tvmc import (HEUN, JASTROW, LJPH, MIDPOINT, PREC_FP64, PREC_MFMA, PROPOSAL_FLIP, PROPOSAL_LEARNED, RBM,  # noqa: F401
                   SIGMA_MINUS, SIGMA_PLUS, SIGMA_Z, Context, Problem, TvmcError, make_config, n_params,
                   unpack_samples)
