"""Back-and-forth optimal transport (quadratic cost, uniform 2D/3D grids) on MI355X.

The compute path is the HIP library ``libbfm.so`` built from ``csrc/``; the
Python module :mod:`paper_1905_12154_amd.bfm` marshals arguments into its C ABI.
Importing this package loads nothing; the library is opened on first use.
"""
__all__ = ["bfm", "workloads"]
