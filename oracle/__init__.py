"""FP64 CPU oracle for the deep-FBSDE hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this package; the product
library never does, and it shares no code with it.
"""
