"""CPU oracle for the RNS-CKKS hot path of FHEON's encrypted CNN layers.

TEST INFRASTRUCTURE ONLY: a plain, slow, obviously-correct reference used by
the test suite, the smoke check and the benchmark's CPU-baseline leg.  The
GPU library neither imports nor links anything here, and this package imports
nothing from the GPU library.
"""
