"""MI355X-native Bayer-domain block-matching motion estimation and feature warp.

Submodules are imported on demand: ``synth`` (seeded synthetic inputs, no
method arithmetic) and ``me`` (the ctypes binding of the HIP library).
"""
__all__ = ["me", "synth"]
