"""PLV / iPLV / ciPLV on MI355X (gfx950): unit-phasor normalisation and one
Hermitian Gram contraction G = U U^H / T on MFMA, behind the C ABI of
include/plv.h (libplv.so, built in-tree by ``paper_1710_08037_amd.build``).

The torch-facing calls live in ``api``; importing this package does not load
the library, the first call does, and raises if it has not been built.
"""
from . import _abi  # noqa: F401

__all__ = ["from_analytic", "from_analytic_noalloc", "from_analytic_batch", "from_real", "from_real_batch", "coherence", "coherence_batch",
           "over_trials", "backward_batch", "coherence_stft", "coherence_stft_batch",
           "PLVFunction", "plv_metrics", "timing_enable", "timing_read", "timing_list", "autotune", "autotune_batch", "tile_edge",
           "set_tile_edge"]


def __getattr__(name):
    if name in __all__:
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
