"""CPU oracle for the level-by-level k-d tree build (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU library.
"""
from .kd_oracle import *  # noqa: F401,F403
