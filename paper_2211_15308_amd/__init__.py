"""MI355X-native solver for -K Delta x + mu^{-1} (-Delta_Gamma)^{-1/2} x = b (Kuchta, arXiv 2211.15308).

The compute path lives in libfdd.so (HIP kernels for gfx950 behind the C ABI of include/fdd.h);
this package is its Python binding.
"""
from .fdd import (FDD_E_ARG, FDD_E_BREAKDOWN, FDD_E_NONFINITE, FDD_E_RA, FDD_E_STATE,  # noqa: F401
                  FDD_E_WORKSPACE, FDD_FP64, FDD_MIXED, FDD_NOT_CONVERGED, FDD_OK, FDD_RA_OPERATOR,
                  FDD_RA_PRECOND, Batch, Cnn, DarcyStokes, FddError, Problem, RationalTable,
                  build_rational_pc, ds_opts_default, load, opts_default, pack_params, precond_apply, schur_apply, setup_darcy_stokes, setup_hdiv, setup_mesh,
                  setup_model, solve,
                  solve_batched, unpack_params)
