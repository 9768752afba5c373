"""fovol: foveated sparse direct volume rendering + neural reconstruction on MI355X.

The compute path is libfovol.so (hand-written HIP for gfx950 behind a C ABI,
``include/fovol.h``); :mod:`paper_2209_09965_amd.binding` is its thin Python
binding.  Importing the binding without the built library raises.
"""
__all__ = ["binding"]
