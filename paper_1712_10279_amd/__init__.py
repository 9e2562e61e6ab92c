"""MI355X-native (gfx950, HIP) solver for vector-valued L1 optimal mass
transport on a regular 2-D grid, after Ryu, Chen, Li and Osher
(arXiv 1712.10279).

The compute path is ``libomt.so`` (HIP kernels behind the C ABI declared in
``include/omt.h``); :mod:`paper_1712_10279_amd.omt` is the Python binding.
The binding loads the library on first use and raises if it is missing.
"""
__all__ = ["omt", "inputs"]
