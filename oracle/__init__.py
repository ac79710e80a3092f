"""CPU oracle for multiple-double polynomial evaluation and differentiation.

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and
the benchmark's CPU-baseline leg, never by the product path.
"""
