"""MI355X-native (gfx950) transit-model hot path of PyTransit (Parviainen 2015).

The model runs in libpthip.so (HIP kernels behind the C ABI of
include/pthip.h); ``paper_1504_07433_amd.pthip`` is its Python binding and
``paper_1504_07433_amd.workloads`` the seeded synthetic inputs.
"""
__all__ = ["workloads", "pthip"]
