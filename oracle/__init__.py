"""FP64 CPU oracle for the coupled Yee-FDTD / quantum-emitter step.

Test infrastructure only: the test-suite, the package smoke check and the
CPU-baseline leg of the benchmark use it.  The product path never imports it.
"""
