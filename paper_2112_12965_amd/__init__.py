"""MI355X-native AB-join (matrix-profile inter-similarity join) for gfx950.

The compute path is the C-ABI HIP library ``libabjoin.so`` (built from
``csrc/`` by ``paper_2112_12965_amd.build``); ``paper_2112_12965_amd.abjoin``
is the thin ctypes binding over it.  ``synth`` draws seeded synthetic inputs.
Importing the package does not load the library.
"""
