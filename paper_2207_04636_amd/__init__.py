"""Robust-pseudospectral occ-RI exchange for periodic Gaussian basis sets on
AMD Instinct MI355X (gfx950).

The computation lives in the HIP library ``librps.so`` (C ABI in
``include/rps.h``); this package only loads it and marshals arguments.
"""
from .binding import (Batch, Context, RpsError, build_batched, exchange_energy, load, madelung_constant,  # noqa: F401
                      PREC_FP64, PREC_FP32, PREC_BF16X3, SELECT_VORONOI, SELECT_GLOBAL,
                      VARIANT_RPS, VARIANT_PS, VARIANT_THC, BATCH_AUTOTUNE, BATCH_BRANCHES, EXPORTS, LIB_PATH)

__all__ = ["Batch", "Context", "RpsError", "build_batched", "exchange_energy", "load", "madelung_constant", "EXPORTS",
           "LIB_PATH"]
