"""CPU oracle (FP64) for the Strang-preconditioned all-at-once BVM solve.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import anything under ``oracle/``.  The
product path (``paper_1305_6653_amd``) never imports it, shares no code with it, and
fails loudly when its HIP library is missing.
"""
from .fde import *  # noqa: F401,F403
