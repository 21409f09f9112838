"""FP64 CPU oracle of the mass-spring method.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, the package smoke check and
the benchmark's CPU-baseline leg, never by the GPU library or its binding.
"""
