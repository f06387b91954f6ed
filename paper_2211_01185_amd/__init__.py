"""MI355X-native particle-side hot path of unresolved CFD-DEM.

The compute path is the HIP library ``lib/libcfddem.so`` (C ABI declared in
``include/cfddem.h``); ``paper_2211_01185_amd.cfddem`` is its thin ctypes
binding.  ``paper_2211_01185_amd.synth`` draws seeded synthetic workloads.
Importing the package itself loads nothing.
"""
__version__ = "0.1.0"
