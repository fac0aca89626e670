"""MI355X-native kernel-independent FMM evaluate for the 3D Laplace kernel.

Importing the package loads nothing native; ``paper_2604_19243_amd.kifmm``
binds the C-ABI library ``libkifmm_mi355x.so`` (built in-tree) and raises if
it is missing.
"""

__all__ = ["workloads", "kifmm"]
