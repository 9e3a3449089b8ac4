"""Fast (polyphase) Haar wavelet transform for AMD Instinct MI355X (gfx950).

The work is done by ``libhaar.so`` (hand-written HIP kernels behind a C ABI,
declared in ``include/haar.h``); this package is its Python binding:

* ``_abi``      -- one ctypes function per C entry point (same names);
* ``transform`` -- torch tensors in/out: fwd1d, inv1d, fwd2d, inv2d, tune_*;
* ``autograd``  -- HaarFwd1D/2D, HaarInv1D/2D autograd Functions;
* ``plan``      -- batched transforms of uneven sizes (persistent launches).
"""
from ._abi import HaarError, LIB_PATH  # noqa: F401


def __getattr__(name):
    # submodules import torch; keep `import paper_1002_2184_amd` light
    import importlib
    if name in ("transform", "autograd", "plan", "_abi"):
        return importlib.import_module(f".{name}", __name__)
    raise AttributeError(name)
