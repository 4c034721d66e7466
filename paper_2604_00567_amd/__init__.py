"""MI355X-native batched power-of-two FFT with the dual-select 6-FMA butterfly.

The compute path is the HIP library ``libdsfft.so`` (built from ``csrc/``) behind
the C ABI declared in ``include/dsfft.h``; ``binding`` marshals arguments to it
with ctypes.  Nothing is loaded at package import: import ``binding`` for the
library, ``inputs`` for the seeded synthetic data (which needs no library).
"""
