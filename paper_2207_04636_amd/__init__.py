"""Robust-pseudospectral occ-RI exchange for periodic Gaussian basis sets on
AMD Instinct MI355X (gfx950).

The computation lives in the HIP library ``librps.so`` (C ABI in
``include/rps.h``); this package only loads it and marshals arguments.
"""
from .binding import (Batch, Context, RpsError, build_batched, exchange_energy, load, madelung_constant,  # noqa: F401
                      PREC_FP64, PREC_FP32, PREC_BF16X3, SELECT_VORONOI, SELECT_GLOBAL,
                      VARIANT_RPS, VARIANT_PS, VARIANT_THC, BATCH_AUTOTUNE, BATCH_BRANCHES, EXPORTS, LIB_PATH,
                      PTRS_HOST, PTRS_DEVICE, RPS_OK, RPS_ERR_ARG, RPS_ERR_SHAPE, RPS_ERR_NOMEM, RPS_ERR_NOT_PD,
                      RPS_ERR_DEVICE, RPS_ERR_STATE)
from . import binding  # noqa: F401

__all__ = ["Batch", "Context", "RpsError", "build_batched", "exchange_energy", "load", "madelung_constant", "EXPORTS",
           "LIB_PATH"]
