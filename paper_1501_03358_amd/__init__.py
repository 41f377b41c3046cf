"""MI355X-native recycling Krylov solvers (rGCROT, rBiCGStab, hybrid) for
sequences of structured-grid pressure-Poisson systems.  The compute path is
the HIP library libkrs.so (C-ABI in include/krs.h); `krs` is its binding."""
