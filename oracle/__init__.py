"""FP64 CPU oracle of the KFVM-WENO right-hand side (test infrastructure only).

Only tests/, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  It shares no code with the GPU library.
"""
