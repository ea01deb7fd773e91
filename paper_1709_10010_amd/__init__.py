"""MI355X-native plane-wave H*psi and block-Davidson (HIP kernels for gfx950).

The compute path lives in ``libpwhip.so`` (C ABI, ``include/pw_api.h``);
this package only marshals arguments to it (``_lib``) and builds problems
from synthetic cells (``problems``).
"""
from ._lib import *  # noqa: F401,F403
from ._lib import LIB, PwError, Problem  # noqa: F401
