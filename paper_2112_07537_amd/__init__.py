"""MI355X-native hot path of the wavelet-adaptive block-structured grid method
of Gillis & van Rees (MURPHY, arXiv 2112.07537): a C-ABI HIP library
(libmr.so, include/mr.h) with a thin ctypes binding (``mr``) and seeded
synthetic workloads (``workloads``)."""
