"""CPU oracle for the Q-adic transform path (test infrastructure only).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package; the product library never does.
"""
from . import gf  # noqa: F401
