"""Pinv-Recon hot path on MI355X: regularised pseudoinverse of the MRI
encoding matrix by the Cholesky route, built and applied by HIP kernels for
gfx950 behind a C-ABI library (libpinv.so).

Importing the package loads nothing; `paper_2410_06129_amd.pinv` loads the
library and raises if it is missing.
"""
__all__ = ["synth", "pinv"]
