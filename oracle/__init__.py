"""Serial double-precision CPU reference of the parallel Metropolis sweeps.

TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
CPU-baseline leg of the benchmark; the GPU library never imports it.
"""
