"""CPU oracle for the cyclic autocorrelation tables (FP64 NumPy, mpmath).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, the graft entry's smoke check
and the benchmark's CPU-baseline leg, never by the product path.  It shares no
code with the HIP library.
"""
