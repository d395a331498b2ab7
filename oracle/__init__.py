"""FP64 CPU oracle for the mesh-transform renderer.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke``
and the CPU-baseline leg of ``bench.py``.  It shares no code with the GPU
library in ``paper_2303_10440_amd`` and neither imports the other.
"""
