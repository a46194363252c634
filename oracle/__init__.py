"""FP64 CPU oracle of the FRE LBM step (test infrastructure only).

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
may import this package.  It shares no code with the GPU library.
"""
