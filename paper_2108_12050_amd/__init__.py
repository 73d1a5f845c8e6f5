"""MI355X-native scale-space LoG focus detector (MHFD, arXiv 2108.12050).

The detector runs in HIP kernels for gfx950 (``libmhfd.so``, C ABI in
``include/mhfd.h``).  Importing the package loads nothing; the first call
that needs the library loads it and raises if it is missing.
"""
from ._lib import MHFDError, MHFDLibraryError  # noqa: F401


def __getattr__(name):
    if name in ("Plan", "Detection", "split_blobs", "FocusScore", "focus_score",
                "stretch_levels"):
        from . import api
        return getattr(api, name)
    if name in ("BatchRunner", "detect_batched"):
        from . import batch
        return getattr(batch, name)
    raise AttributeError(name)
