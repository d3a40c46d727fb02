"""MI355X (gfx950) inpainting path for diminished-reality privacy.

``Inpainter(cfg, weights)`` wraps one context of the HIP library ``libdrinpaint.so``
(C ABI in include/drinpaint.h); ``inpaint(...)`` is the one-shot form.  The package is
imported lazily so that the weight-blob helpers work without a GPU.
"""
__all__ = ["Inpainter", "inpaint"]


def __getattr__(name):
    if name in ("Inpainter", "inpaint"):
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
