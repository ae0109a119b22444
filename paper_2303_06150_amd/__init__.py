"""MI355X-native docking hot path (LiGen-style virtual screening).

``lg`` is the thin binding of the C ABI in ``include/lg.h``; the kernels live in
``csrc/`` and are built by ``build.py`` into ``liblg.so`` (gfx950).
"""
from . import lg  # noqa: F401

__all__ = ["lg"]
