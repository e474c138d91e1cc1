"""MI355X library for the RK2 substep of the low-Mach variable-density
pseudospectral method (Reuter, Oliver & Moser).

Modules: ``lmvd`` (ctypes binding of the HIP library), ``workloads`` (seeded
synthetic inputs), ``build`` (compiles ``_lmvd.so`` for gfx950)."""
