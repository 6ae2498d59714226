"""MI355X-native D2Q9 finite-volume kinetic steps (DUGKS and BKG) of
Zhu, Wang & Guo (arXiv 1511.00242).

The compute path is the C-ABI library ``liblbfv.so`` (hand-written HIP kernels
for gfx950, declared in ``include/lbfv.h``); :mod:`.lbfv` is its thin ctypes
binding.  Importing this package does not load the library.
"""
