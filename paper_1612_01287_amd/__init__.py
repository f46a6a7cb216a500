"""MI355X (gfx950) implementation of the R-SLB time step for massless particles
(Ambrus & Blaga, arXiv:1612.01287): a HIP C-ABI library (librsl.so, include/rsl.h)
and a thin ctypes binding (rsl.py) that uses torch only for device memory and
streams."""
