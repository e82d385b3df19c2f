"""PackUV-GS differentiable splatting on MI355X (gfx950).

The compute path is the HIP library ``libpackuvgs.so`` (C ABI in
``include/packuv_gs.h``); this package holds its ctypes binding (``_abi``),
the buffer/call-chain driver and autograd wrapper (``pipeline``), the
autotuner (``autotune``) and the build script (``build``).
"""
from . import _abi as abi  # noqa: F401

__all__ = ["abi", "Renderer", "PackUVRender"]


def __getattr__(name):
    if name in ("Renderer", "PackUVRender"):
        from . import pipeline
        return getattr(pipeline, name)
    raise AttributeError(name)
