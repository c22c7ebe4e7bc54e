"""Surrogate-matrix isogeometric assembly on MI355X (gfx950).

Importing the package is cheap: the HIP library is loaded by
``paper_1904_06971_amd.igs`` on first use, and fails loudly when it is missing.
"""
__all__ = ["igs", "workloads", "autograd"]
__version__ = "0.1.0"
