"""MI355X-native multi-channel Lenia step with localized genotypes.

The compute path lives in the HIP library ``liblenia.so`` behind the C ABI of
``include/lenia.h``; this package holds its ctypes binding (``lenia``), the
checkpointed autograd wrapper (``autograd``) and the seeded input generators
(``inputs``).  Importing the package does not load the library; the first call
that needs it does, and raises if it is missing.
"""
__all__ = ["inputs"]
