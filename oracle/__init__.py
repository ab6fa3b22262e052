"""CPU oracle for the pseudo-spectral Navier-Stokes step (test infrastructure).

Only the tests, the package's smoke check and the benchmark's CPU-baseline leg
may import this package.  The GPU library never imports, links or calls it.
"""
from .spectral_ns import *  # noqa: F401,F403
from .implicit_midpoint import *  # noqa: F401,F403
from .mlp import *  # noqa: F401,F403
from .triads import *  # noqa: F401,F403
from .surrogate_data import *  # noqa: F401,F403
from .spectral_ns import __all__ as _a
from .implicit_midpoint import __all__ as _b
from .mlp import __all__ as _c
from .triads import __all__ as _d
from .surrogate_data import __all__ as _e

__all__ = list(_a) + list(_b) + list(_c) + list(_d) + list(_e)
