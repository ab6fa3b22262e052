"""CPU oracle for the pseudo-spectral Navier-Stokes step (test infrastructure).

Only the tests, the package's smoke check and the benchmark's CPU-baseline leg
may import this package.  The GPU library never imports, links or calls it.
"""
from .spectral_ns import *  # noqa: F401,F403
from .implicit_midpoint import *  # noqa: F401,F403
from .mlp import *  # noqa: F401,F403
from .triads import *  # noqa: F401,F403
from .spectral_ns import __all__ as _a
from .implicit_midpoint import __all__ as _b
from .mlp import __all__ as _c
from .triads import __all__ as _d


def surrogate_pairs(*args, **kwargs):
    """oracle.surrogate_data.surrogate_pairs (imported on first use, so that
    `python -m oracle.surrogate_data` runs the module once)."""
    from .surrogate_data import surrogate_pairs as f
    return f(*args, **kwargs)


__all__ = list(_a) + list(_b) + list(_c) + list(_d) + ["surrogate_pairs"]
