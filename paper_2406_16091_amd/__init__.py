"""MI355X-native grid-binned cutoff pair interactions (arXiv 2406.16091).

The compute path is the C-ABI library ``libpi.so`` (hand-written HIP for
gfx950) declared in ``include/pi.h``; :mod:`paper_2406_16091_amd.pi` is its
thin ctypes binding.  :mod:`paper_2406_16091_amd.synth` draws the seeded
synthetic systems.  Importing this package loads nothing; the binding loads
the library on first use and raises if it is missing.
"""
