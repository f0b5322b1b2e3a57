"""MI355X (gfx950) implementation of the DiaQ state-vector hot path.

The compute lives in ``libdiaq_hip.so`` (hand-written HIP kernels behind the
C ABI declared in ``include/diaq.h``); :mod:`.diaq` is a thin ctypes binding
with the same names.  Importing this package loads nothing; the library is
opened on first use of :mod:`.diaq`.
"""
__all__ = ["inputs", "diaq"]
