"""MI355X-native treecode hot path (Barnes-Hut style, §3.1 of Duy,
Yamazaki & Oyanagi): Morton keys, radix sort, quad/oct-tree, FP64 moments,
a group walk with LDS-staged interaction lists and an FP32 force loop, all
hand-written HIP kernels for gfx950 behind the C-ABI of ``include/tc.h``.

The GPU library is loaded lazily by :mod:`paper_1211_2293_amd.treecode`;
importing the package itself needs neither a GPU nor the built library.
"""
__all__ = ["treecode", "workloads"]
