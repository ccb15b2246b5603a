"""MI355X-native multislice (CSSI reflection geometry) forward model and gradient.

The compute path is the HIP library ``libmsl.so`` (C ABI declared in
``include/msl.h``); ``paper_2212_01253_amd.msl`` is its thin ctypes binding.
Importing the package does not load the library; ``msl.lib()`` does, and it
raises if the library is missing.
"""
__all__ = ["msl", "synth"]
