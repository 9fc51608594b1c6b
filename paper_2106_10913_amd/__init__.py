"""MI355X-native AWG-preconditioned CG (Gouarin & Spillane, arXiv 2106.10913).

The solver lives in ``libawg.so`` (HIP kernels for gfx950 behind the C ABI of
``include/awg.h``); :mod:`paper_2106_10913_amd.awg` is a thin ctypes binding
that marshals torch device tensors into it.
"""
