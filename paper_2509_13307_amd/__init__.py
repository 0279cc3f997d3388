"""MI355X-native batched likelihoods and nested slice sampling.

Hot path of GPU-accelerated nested sampling with neural emulators
(Lovick et al., arXiv:2509.13307): emulator MLP -> [Limber projection with
nuisances] -> Gaussian chi^2 for thousands of walkers, the slice-step kernel
and the FP64 evidence accumulator, in hand-written HIP for gfx950 behind the
C ABI of include/ns.h.  This package is the thin Python binding.
"""
from ._capi import NSError, PRECISIONS, LIB_PATH  # noqa: F401


def Model(*args, **kwargs):
    """Create a device-resident model (see paper_2509_13307_amd.model.Model)."""
    from .model import Model as _M
    return _M(*args, **kwargs)
