"""MI355X-native nested-dissection Cholesky factorization and solve of
symmetric positive-definite block-tridiagonal matrices (arXiv 2601.03754).

The compute path is the C-ABI library ``libbtc.so`` (HIP kernels for gfx950,
see ``include/btc.h``); ``paper_2601_03754_amd.btc`` is its thin Python
binding.  The library is loaded on first use, and every entry point raises if
it is missing: there is no CPU fallback.
"""
__all__ = ["inputs"]
