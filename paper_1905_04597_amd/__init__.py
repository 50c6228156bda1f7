"""glbm: Gaussian lattice Boltzmann hierarchy (arXiv:1905.04597) on MI355X.

The compute path is the HIP library ``libglbm.so`` (C-ABI declared in
``include/glbm.h``); :mod:`paper_1905_04597_amd.glbm` is its ctypes binding,
with PyTorch used only for device memory and streams.  Importing this
package does not load the library; :func:`paper_1905_04597_amd.glbm.load`
does, and raises if it is missing.
"""

__all__ = ["glbm", "workloads"]
