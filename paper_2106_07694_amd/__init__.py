"""MI355X-native coupled lattice-Boltzmann + WENO step (arXiv 2106.07694).

The compute path is the C-ABI library ``liblbw.so`` (hand-written HIP for
gfx950, declared in ``include/lbw.h``); ``paper_2106_07694_amd.lbw`` is its
thin ctypes binding.  Importing the package does not load the library.
"""
__all__ = ["workloads", "lbw"]
