"""MI355X (gfx950) library for the unfitted boundary algebraic equation method with
free-space lattice Green's functions (arXiv 2502.05507).

The compute path is the C-ABI shared library libbae.so (HIP kernels + C++ host code,
declared in include/bae.h); this package is a thin ctypes binding with the same names.
Importing the package does not load the library; the first call does, and it fails
loudly when libbae.so has not been built (python -m paper_2502_05507_amd.build).
"""
from .binding import (BaeError, Batch, Context, Server, lgf_table, lgf_table_noalloc, lgf_table_size,  # noqa: F401
                      load_library,
                      PREC_FP64, PREC_FP32, PREC_FFT, SOLVE_FP64, SOLVE_FP32_REFINED, SOLVE_FFT, LAYER_DOUBLE, LAYER_SINGLE, LAYER_DIRECT, KINDS)
