"""MI355X-native randomized Cholesky QR (Balabanov, arXiv 2210.09953).

Thin ctypes binding over librcholqr.so (include/rcholqr.h).  Every step of
the factorisation runs in the library's HIP kernels; this module only
allocates tensors with PyTorch, passes raw device pointers and the current
HIP stream, and checks return codes.  If the library is not built the calls
raise: there is no fallback implementation.

Matrices are column-major: an (m, n) tensor with stride (1, ld), ld >= m.
"""
from .binding import (GAUSSIAN, RADEMACHER, COUNTSKETCH, SRHT, IDENTITY_TESTONLY, F64, F32, MIXED,
                      LibraryMissing, RCholQRError, lib, lib_path,
                      workspace_bytes, factor, sketch, debug_theta, trsm,
                      status, error_string, fortran, empty_fortran, PHASES,
                      profile_enable, profile_read, backward, BatchedFactor, Problem, ColumnQR,
                      device_copy, reduced, rr, factor_noalloc, noalloc_status,
                      noalloc_max_bytes, BatchedEngine, BATCH_INVALID, init)
from .autograd import RCholQR2, rcholqr2

__all__ = ["GAUSSIAN", "RADEMACHER", "COUNTSKETCH", "SRHT", "IDENTITY_TESTONLY", "F64", "F32", "MIXED",
           "LibraryMissing", "RCholQRError", "lib", "lib_path",
           "workspace_bytes", "factor", "sketch", "debug_theta", "trsm",
           "status", "error_string", "fortran", "empty_fortran", "PHASES",
           "profile_enable", "profile_read", "backward", "RCholQR2", "rcholqr2", "device_copy",
           "BatchedFactor", "Problem", "ColumnQR", "reduced", "rr", "factor_noalloc",
           "noalloc_status", "noalloc_max_bytes", "BatchedEngine", "BATCH_INVALID", "init"]
