"""MI355X (gfx950) ATRG / triad-ATRG coarse-graining behind a small C ABI.

The product path is the shared library ``libtrg.so`` built from ``csrc/``;
this package only marshals arguments to it (ctypes).  It raises if the
library is missing: there is no CPU fallback.
"""
from .binding import (Solver, Batch, Graph, TrgError, load_library, selftest_gemm, selftest_tsqr, selftest_permute, selftest_svd, selftest_eigh,
                      selftest_pchol, selftest_gram_eig,
                      selftest_sketch, qr, qr_noalloc, FP64, FP32, BF16X3, BF16X6, SVD_SKETCH, SVD_EXACT, MODEL_ISING,
                      T_PHI, T_PSI, T_SIGMA, T_RESPLIT, TAN_BETA, TAN_H, METHOD_ATRG, METHOD_TRIAD)

__all__ = ["Solver", "Batch", "Graph", "TrgError", "load_library", "selftest_gemm", "selftest_tsqr", "selftest_permute", "selftest_svd", "selftest_eigh",
           "selftest_pchol", "selftest_gram_eig",
           "selftest_sketch", "qr", "qr_noalloc", "FP64", "FP32", "BF16X3", "BF16X6", "SVD_SKETCH", "SVD_EXACT", "MODEL_ISING",
           "T_PHI", "T_PSI", "T_SIGMA", "T_RESPLIT", "TAN_BETA", "TAN_H",
           "METHOD_ATRG", "METHOD_TRIAD"]
