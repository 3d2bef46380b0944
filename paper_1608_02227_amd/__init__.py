"""MI355X-native dual-smoothing (P-APG) convex-regression fits.

Importing the package loads nothing native; ``paper_1608_02227_amd.cr`` binds the C-ABI library
``libcr.so`` (HIP kernels for gfx950) on first use and raises if it is missing.
"""
__all__ = ["cr", "workloads"]
