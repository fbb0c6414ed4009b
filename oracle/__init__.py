"""CPU oracle for norm-ranging LSH -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the bench's CPU-baseline leg
may import this package.  The product library never does.
"""
from .oracle import *  # noqa: F401,F403
