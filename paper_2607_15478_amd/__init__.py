"""MI355X-native exact ParDTW (parallelized diagonal dynamic time warping).

The compute path lives in ``libpardtw.so`` (hand-written HIP for gfx950 behind
a C ABI declared in ``include/pardtw.h``). ``paper_2607_15478_amd.pardtw`` is
the thin ctypes binding; it is imported lazily so that the seeded input
generators in ``paper_2607_15478_amd.synth`` load without a GPU library.
"""
__all__ = ["synth"]
