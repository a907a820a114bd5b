"""MI355X-native Triangle p-1-Reduction and uniform edge sampling (Slim Graph).

Submodules:
  * ``slim``     -- ctypes binding of the C-ABI library ``libslim.so`` (HIP, gfx950)
  * ``graphgen`` -- seeded synthetic input graphs (G(n,q), R-MAT)
"""
__all__ = ["slim", "graphgen"]
