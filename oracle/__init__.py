"""FP64 CPU oracle for the SU(2) heat bath.

TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the benchmark's
CPU-baseline leg.  The GPU library never imports, links or calls anything here.
"""
