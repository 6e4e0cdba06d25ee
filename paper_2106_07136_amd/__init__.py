"""MI355X-native Bayesian Dense Inverse Search (BDIS) stereo.

Paper: J. Song, Q. Zhu, J. Lin, M. Ghaffari, "Bayesian dense inverse searching
algorithm for real-time stereo matching in minimally invasive surgery",
arXiv 2106.07136.  The hot path runs as hand-written gfx950 HIP kernels in
``libbdis.so`` behind the C ABI of ``include/bdis.h``; ``bdis`` is its thin
Python binding (torch tensors supply device memory and streams).
"""
__all__ = ["bdis", "synth"]
