"""MI355X-native DD-alpha-AMG solver for the twisted-mass clover Wilson operator.

The compute path is the HIP library libtmamg.so (include/tmamg.h); this
package only marshals arguments to it (see binding.py) and builds it
(build.py).
"""
from .binding import (Solver, Params, Info, default_params, load, TmamgError,  # noqa: F401
                      FP64, MIXED, STORE_FP64, STORE_FP32, STORE_BF16, STORE_FP16,
                      OP_D64, OP_D32, OP_PROLONG, OP_RESTRICT, OP_DC, OP_SAP, OP_PREC, OP_COARSEST, EXPORTS,
                      OP_SCHUR64, OP_SCHUR32, OP_DDAG64, OP_DDAG32, OP_DCND, OP_SAPND, check_field, torch_allocator,
                      K_DSLASH32, K_DSLASH64, K_SAP0, K_RESTRICT0, K_PROLONG0, K_DC1, K_DC2, K_SAP1, K_COPY, K_SCHUR32,
                      TUNE_COARSE_APPLY, TUNE_SAP1, TUNE_RESTRICT0, TUNE_PROLONG0, TUNE_SAP0,
                      tune_load, tune_save, tune_set, tune_get, tune_entries, tune_clear)
from .autograd import FermionAction, fermion_action  # noqa: F401,E402
