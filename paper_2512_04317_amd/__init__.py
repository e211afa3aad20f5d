"""MI355X (gfx950) MX-scaled mixed-precision 2D FFT.

The transform runs in hand-written HIP kernels behind the C ABI declared in
``include/mxfft.h`` (shared library ``libmxfft.so`` in this package).  The
Python binding in :mod:`paper_2512_04317_amd.mxfft` only marshals arguments.
"""
