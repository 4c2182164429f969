"""CPU oracle for the TaCo query stage -- TEST INFRASTRUCTURE ONLY.

Used by the tests, the smoke check and the benchmark's CPU-baseline leg to
define expected results; never by the product.  See ``oracle.oracle``.
"""
