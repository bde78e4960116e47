"""MI355X (gfx950) KFVM-WENO right-hand side: HIP kernels behind a C-ABI
(include/kfvm.h), with a thin ctypes binding (`paper_2401_16543_amd.kfvm`)."""
