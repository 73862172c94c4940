"""Differentiable CSR sparse kernels (SpMV, SpMM, SpGEMM, triangular solve)
for AMD Instinct MI355X (gfx950), after arXiv 2212.05159.

Importing the package loads nothing native; ``paper_2212_05159_amd.capi``
loads the HIP library on first use and fails loudly if it is missing.
"""
__all__ = ["gen"]
