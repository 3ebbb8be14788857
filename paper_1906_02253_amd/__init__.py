"""MI355X-native Kalman-filter track fit and combinatorial track finding
(arXiv:1906.02253, mkFit), hand-written HIP kernels for gfx950 behind the C ABI
in include/kf.h.  This package is the thin Python binding; importing it loads
libkfmi.so and fails if the library is not built.
"""
from .binding import (Context, Tracks, Hits, KFError, lib, round_ld, PREC_MIXED, PREC_FP32,
                      PREC_FP64, INIT_MLP, NO_MATERIAL, PER_LAYER, CLEAN_SEEDS,
                      REMOVE_DUPLICATES, ST_OK, ST_UNREACHABLE,
                      ST_NOCONV, ST_FALLBACK, ST_NONPD, ST_NAN, ST_BADINPUT, ST_DUPLICATE, ST_DUPTRACK,
                      LIB_PATH)

__all__ = ["Context", "Tracks", "Hits", "KFError", "lib", "round_ld", "PREC_MIXED", "PREC_FP32",
           "PREC_FP64", "INIT_MLP", "NO_MATERIAL", "PER_LAYER", "CLEAN_SEEDS",
           "REMOVE_DUPLICATES", "ST_OK", "ST_UNREACHABLE",
           "ST_NOCONV", "ST_FALLBACK", "ST_NONPD", "ST_NAN", "ST_BADINPUT", "ST_DUPLICATE", "ST_DUPTRACK",
           "LIB_PATH"]
