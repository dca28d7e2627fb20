"""MI355X-native CG-SENSE: multicoil Cartesian MRI encoding on one GPU.

The compute path is a HIP library for gfx950 (``csrc/``) behind a C ABI
(``include/sense.h``); :mod:`.sense` is its thin ctypes binding over torch
device memory and streams.  :mod:`.synth` draws seeded synthetic inputs.
Importing the package does not load the library; the first call does, and
fails loudly if it has not been built.
"""

__all__ = ["synth", "sense"]
