"""MI355X-native hypersingular BEM on polygonal multiscreens with a two-level substructuring
preconditioned CG solve.  The compute path lives in the HIP shared library ``libbem.so``
(C-ABI declared in include/bem.h); this package only marshals arguments to it."""
