"""MI355X-native (gfx950) time-stepped 3D elastic velocity-stress finite differences
(arXiv 2112.15071): hand-written HIP kernels behind a C ABI (include/fd3d.h), with
torch supplying device memory and streams.

The HIP library is required: importing ``Simulator`` loads ``libfd3d.so`` and fails
loudly if it is missing.  There is no CPU fallback.
"""
__version__ = "0.1.0"


def __getattr__(name):
    if name in ("Simulator", "make_opts", "make_source", "FIELDS", "upsample", "forward_static"):
        from . import simulator

        return getattr(simulator, name)
    raise AttributeError(name)
