"""FP64 CPU reference ("oracle") for the exact softened all-pairs gravity sum.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
bench's CPU-baseline leg, never by the product path.  It shares no code with
the HIP library and imports nothing from it.
"""
