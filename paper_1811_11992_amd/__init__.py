"""MI355X-native Newton hot path of a fully implicit in-situ-combustion simulator.

The GPU library (``libisc.so``, HIP for gfx950, C-ABI declared in
``include/isc.h``) is loaded on first use by :mod:`paper_1811_11992_amd.isc`;
importing the package itself needs no GPU.
"""
