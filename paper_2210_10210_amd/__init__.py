"""EFGP on MI355X: equispaced-Fourier Gaussian process regression with
hand-written gfx950 HIP kernels behind a C ABI (include/efgp.h).

The binding lives in ``paper_2210_10210_amd.capi``; importing it loads the
HIP library and fails if it is not built.  This package import itself is
light so that the build step can run without a GPU.
"""


def load_binding():
    """Import and return the ctypes binding (loads libefgp.so)."""
    from . import capi as _c
    return _c
