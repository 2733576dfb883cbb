"""MI355X-native FFT phase-field twin-propagation step.

The compute path is the HIP library ``libpftwin.so`` (C ABI declared in
``include/pf.h``); ``binding`` is a thin ctypes layer over it and loads it on
first use, failing loudly if it has not been built. ``inputs`` holds the
seeded synthetic workload generators.
"""
