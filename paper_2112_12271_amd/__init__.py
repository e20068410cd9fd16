"""hdMD hot path on MI355X: d-dimensional cell binning, 3^d-stencil Verlet
lists with a skin, WCA / harmonic pair forces, velocity Verlet and FIRE 2.0,
as hand-written HIP kernels behind a C ABI (``include/hdmd.h``).

The native library is loaded lazily by :mod:`paper_2112_12271_amd.hdmd`; this
package import itself touches no GPU.
"""
__all__ = ["inputs"]
