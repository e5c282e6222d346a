"""Split-format complex DFT for AMD MI355X (gfx950).

Batched N-point DFT on separate real and imaginary planes,
yr = C xr + S xi and yi = C xi - S xr, evaluated through the Kronecker
factorisation of Cariow (arXiv 2504.07264, Section III, eq. 6) by hand-written
HIP kernels behind the C ABI of include/split_dft.h.

The library is loaded on first use; a missing build raises.
"""
from .binding import (FP32, ManyGraph, ManyPlan, Plan, SplitDFTError, cached_plan,  # noqa: F401
                      many_flags, split_dft, split_dft_adjoint, twiddle_table, variant_flag)
from .autograd import SplitDFTFunction, split_dft_autograd  # noqa: F401

__all__ = ["Plan", "ManyPlan", "ManyGraph", "many_flags", "SplitDFTError", "split_dft", "split_dft_adjoint", "split_dft_autograd",
           "SplitDFTFunction", "twiddle_table", "variant_flag", "cached_plan", "FP32"]
