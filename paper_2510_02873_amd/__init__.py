"""MI355X collapse-time library: Python binding of libpino_collapse.so.

Every computation happens in the HIP kernels behind the C ABI of
include/pino_collapse.h; this package only marshals arguments.
"""

from ._abi import (PINO_ABI_VERSION, PINO_CLASSIC, PINO_TABULATED, PINO_CLASSIC_LCDM, PINO_FP64, PINO_MIXED,
                   PINO_SURROGATE, PINO_EVAL_RESET, PINO_EVAL_SYNC, PINO_EVAL_FINALIZE, PINO_OK, PINO_ERR_ARG,
                   PINO_ERR_ALLOC, PINO_ERR_HIP, PINO_ERR_STATE, PINO_ERR_UNSUPPORTED, Config,
                   PinoError, make_item, pino_collapse_init, pino_collapse_eval, pino_collapse_free,
                   pino_collapse_last_error, lib, LIB_PATH, Field)
from .runner import Collapse

__all__ = [
    "PINO_ABI_VERSION", "PINO_CLASSIC", "PINO_TABULATED", "PINO_CLASSIC_LCDM", "PINO_FP64", "PINO_MIXED", "PINO_SURROGATE",
    "PINO_EVAL_RESET", "PINO_EVAL_SYNC", "PINO_EVAL_FINALIZE", "PINO_OK", "PINO_ERR_ARG", "PINO_ERR_ALLOC", "PINO_ERR_HIP",
    "PINO_ERR_STATE", "PINO_ERR_UNSUPPORTED", "Config", "PinoError", "make_item", "pino_collapse_init",
    "pino_collapse_eval", "pino_collapse_free", "pino_collapse_last_error", "lib", "LIB_PATH", "Collapse", "Field",
]
