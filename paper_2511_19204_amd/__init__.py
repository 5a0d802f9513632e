"""MI355X-native hot path of reference-free sampling-based MPC (arXiv 2511.19204).

The compute lives in ``libmppi.so`` (hand-written HIP for gfx950 behind a C ABI,
declared in ``include/mppi.h``); ``paper_2511_19204_amd.mppi`` is the thin ctypes
binding and ``paper_2511_19204_amd.synth`` makes seeded synthetic workloads.
Importing this package loads nothing; the binding loads the library on first use.
"""
__all__ = ["synth"]
