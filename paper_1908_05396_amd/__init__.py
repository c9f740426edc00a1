"""MI355X-native D3Q19 cascaded (central-moment) lattice Boltzmann method for
power-law fluids (arXiv:1908.05396).

The hot path, a fused pull stream-collide kernel with the locally solved
power-law relaxation rate, lives in the HIP library ``libclbm.so`` (C-ABI in
``include/clbm.h``).  This package holds its sources (``csrc/``), the build
step and a thin ctypes binding; importing ``paper_1908_05396_amd.clbm`` fails
if the library has not been built.
"""
__all__ = ["clbm", "build"]
