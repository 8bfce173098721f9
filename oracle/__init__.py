"""FP64 CPU oracle of the regularized colour-gradient LB printing model.

Test infrastructure only: loaded by the tests, the smoke check and the
CPU-baseline leg of the benchmark, never by the GPU library or its binding.
"""
