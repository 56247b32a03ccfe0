"""FP64 CPU oracle for the particle-decomposition SPH hot path.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package; the HIP library and its binding
never do, and nothing here imports them.
"""
