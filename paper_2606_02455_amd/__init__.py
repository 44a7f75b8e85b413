"""MI355X-native batched verification for Langevin Speculative Dynamics.

The compute path is the HIP library ``liblsd.so`` (built from csrc/ for
gfx950) behind the C ABI declared in include/lsd.h; ``lsd`` is its thin
ctypes binding.  ``workloads`` holds the seeded input generators only.
Importing the package does not load the library; ``lsd.load()`` does, and
raises if it is missing.
"""
__all__ = ["workloads", "lsd"]
