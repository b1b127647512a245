"""FP64 CPU oracle of the VP-LBM time step (test infrastructure only).

Only the test suite, the package smoke check and the benchmark's CPU-baseline leg
import this package.  The GPU product path never imports it.
"""
