"""MI355X-native DG diffusion solver for the displacement covariance of the
ensemble average propagator in an axon substrate (arXiv 1907.06191).

The product is the C-ABI library ``libdgd.so`` (include/dgd.h) built from
``csrc/`` with hipcc for gfx950; ``paper_1907_06191_amd.dgd`` is its thin
ctypes binding.  Importing the binding fails loudly when the library has
not been built: there is no CPU fallback.
"""

__all__ = ["dgd"]
