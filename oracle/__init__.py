"""FP64 CPU oracle of the explicit MHD step (test infrastructure only).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark
import this package; the product library never does.
"""
