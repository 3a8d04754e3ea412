"""MI355X (gfx950) DWT pan-sharpening: fused forward-DWT / replace-LL /
inverse-DWT of a PAN image with each MS band (Haar or Daubechies-4 with
periodic wrap), its batched persistent form and its adjoint.

The computation lives in the HIP library ``libdwtfuse.so`` behind the C ABI
of ``include/dwt_fuse.h``; this package only marshals torch tensors into it.
Importing the package does not load the library; the first call does, and
raises if it has not been built.
"""
from ._lib import D4, HAAR, DwtFuseError, LIB_PATH  # noqa: F401


def __getattr__(name):
    # Lazy: the torch-facing API is imported on first use.
    if name in ("fuse", "fuse_batched", "fuse_backward", "fuse_backward_noalloc", "fuse_backward_batched",
                "fuse_multipass", "quality",
                "DwtFuseFn", "Context", "context", "make_items", "make_bwd_items"):
        from . import api

        return getattr(api, name)
    raise AttributeError(name)
