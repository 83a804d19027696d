"""MI355X-native implementation of the per-step hot path of the entropic
multi-relaxation-time two-phase lattice Boltzmann model (Hosseini, Dorschner
& Karlin, arXiv:2201.12404): HIP kernels for gfx950 behind a C ABI
(include/elmrt.h), with a ctypes binding in :mod:`.elmrt`."""
