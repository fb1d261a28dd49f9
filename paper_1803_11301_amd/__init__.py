"""MI355X (gfx950) multiplication of long bit polynomials in GF(2)[x] with
Frobenius partitions in the additive FFT (Chen, Cheng, Kuo, Li, Yang).

The HIP library (``libfpmul.so``, C ABI in ``include/fpmul.h``) is loaded by
``paper_1803_11301_amd.fpmul``; importing this package loads nothing.
"""
__all__ = ["fpmul", "synth"]
