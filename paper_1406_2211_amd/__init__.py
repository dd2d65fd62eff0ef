"""MI355X (gfx950) lattice Boltzmann with operator-split second-order forcing
and fluid-particle coupling (after Schiller, arXiv:1406.2211).

The compute path is the HIP library ``liblbc.so`` (C ABI in ``include/lbc.h``);
``paper_1406_2211_amd.lbc`` is its ctypes binding.  Importing the package does
not load the library; using the binding without a built library raises.
"""
__all__ = ["inputs", "lbc"]
