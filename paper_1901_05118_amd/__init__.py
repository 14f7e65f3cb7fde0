"""MI355X-native EXCMG solver for the 3D biharmonic equation (arXiv:1901.05118).

The numerical work runs in ``libexcmg.so`` (hand-written HIP for gfx950 behind the C ABI in
``include/excmg.h``); ``paper_1901_05118_amd.excmg`` is a thin ctypes binding with the same
names.  There is no CPU fallback: importing the binding fails if the library is not built.
"""
from .excmg import *  # noqa: F401,F403
from .excmg import __all__  # noqa: F401
