"""FP64 CPU oracle (test infrastructure only).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU library.
"""
from .mvrl import *  # noqa: F401,F403
from .mvrl import EPS, ZERO, PERIODIC, SIMULTANEOUS, SEQUENTIAL  # noqa: F401
