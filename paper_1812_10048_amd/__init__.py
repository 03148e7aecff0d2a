"""MI355X-native sub-cluster split/merge sampler for Dirichlet-process mixtures
of multinomials over UMI counts (Duan, Pinto & Xie, arXiv:1812.10048).

The compute path lives in ``libdpmm.so`` (hand-written HIP kernels for gfx950
behind a C ABI, declared in ``include/dpmm.h``); ``paper_1812_10048_amd.dpmm``
is the thin ctypes binding and ``Sampler`` its Python face.  Importing this
package does not load the library; the first use does, and fails loudly if it
has not been built.
"""
import importlib

__all__ = ["Sampler", "DMLogMarginal", "eb_update_beta"]


def __getattr__(name):
    if name in __all__:
        return getattr(importlib.import_module(__name__ + ".sampler"), name)
    raise AttributeError(name)
