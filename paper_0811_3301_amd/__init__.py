"""MI355X-native two-pass DTW nearest-neighbour search (LB_Keogh -> LB_Improved -> banded DTW_p).

The compute path lives in the HIP library ``liblbimp.so`` (C-ABI declared in
``include/lbimp.h``); ``paper_0811_3301_amd.lbimp`` is its thin ctypes binding.
Importing this package loads nothing: ``gen`` (seeded inputs) works without a GPU.
"""
