"""MI355X-native streaming cyclic statistics (cyclic autocorrelation R^a(t) and
its conjugate form) over a grid of cycle frequencies and lags.

The compute path is the HIP library ``libcyclo.so`` (C ABI in
``include/cyclo.h``); :mod:`paper_2405_16911_amd.cyclo` is its thin ctypes
binding.  Importing this package does not load the library.
"""
