"""Enhanced discrete PSO for UAV inspection path planning on MI355X (gfx950).

Submodules:
  dpso    binding of the C ABI (``include/dpso.h``); imports torch
  scenes  seeded synthetic viewpoint / obstacle scenes (numpy only)
  build   hipcc build of ``libdpso.so``
"""
__version__ = "0.1.0"
