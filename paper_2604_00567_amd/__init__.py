"""MI355X-native batched power-of-two FFT with the dual-select 6-FMA butterfly.

The compute path is the HIP library ``libdsfft.so`` (built from ``csrc/``) behind
the C ABI declared in ``include/dsfft.h``; ``binding`` marshals arguments to it
with ctypes.  Nothing is loaded at import time: ``inputs`` (seeded synthetic
data) imports without the library.
"""
__all__ = ["binding", "inputs"]


def __getattr__(name):
    if name == "binding":
        from . import binding
        return binding
    raise AttributeError(name)
