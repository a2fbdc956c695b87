"""MI355X (gfx950) implementation of the ILE marginalized-likelihood step of
arXiv 2210.07912: extrinsic sampling, the mode-decomposed likelihood from the
overlaps Q and U, time marginalization by log-sum-exp, and the FP64
importance-sampling estimate, as HIP kernels behind the C ABI in
``include/rift_ile.h``.  ``ile`` is the Python binding."""

__all__ = ["ile", "build"]
