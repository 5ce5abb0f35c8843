"""MI355X (gfx950) Wilson-Dirac inverter hot path: HIP kernels behind a C ABI.

The library (libwilson.so, built from csrc/ by build.py) applies the Wilson
D-slash, solves the Wilson system by mixed-precision even-odd CG on the
normal equations (single and batched), and applies the Chebyshev sign
function of the overlap kernel.  ``wilson`` is its Python binding.
"""
from . import wilson  # noqa: F401
