"""CPU oracle for the two-level Schwarz preconditioned normal-equations solve.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The library in
``paper_2107_09006_amd`` never imports it, and the two share no code: the only
common dependency is the seeded input generator package ``workloads``.
"""
from .lsq2l_oracle import *  # noqa: F401,F403
