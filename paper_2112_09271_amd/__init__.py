"""dgnp: MI355X (gfx950) DG solver for the charge-conservation Nernst-Planck
equations (arXiv 2112.09271).  The solver lives in libdgnp.so (C ABI in
include/dgnp.h); `paper_2112_09271_amd.dgnp` is its ctypes binding."""
