"""MI355X-native hot path of multigrid low-mode averaging (arXiv:2412.06347).

The computation lives in ``libmglma.so`` (hand-written HIP for gfx950 behind
the C ABI ``include/mglma.h``); ``mglma`` is its ctypes binding, ``synth``
the seeded synthetic inputs, ``build`` the in-tree build.
"""
__all__ = ["mglma", "synth", "build"]
