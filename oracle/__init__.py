"""FP64 CPU oracle for the FDAS hot path (test infrastructure only).

Imported by tests/, __graft_entry__.smoke() and the CPU-baseline leg of bench.py.
The product package never imports it.
"""
from . import fdas64  # noqa: F401
