"""MI355X-native dense GF(2) decomposition (Bertolazzi & Rimoldi, "Fast matrix
decomposition in F2").

The compute path is the C-ABI library ``libgf2.so`` (hand-written HIP kernels
for gfx950, declared in ``include/gf2.h``); :mod:`paper_1209_5198_amd.gf2` is
its thin ctypes binding.  :mod:`paper_1209_5198_amd.synth` generates the seeded
synthetic inputs.  Importing this package does not load the GPU library; the
first call into :mod:`.gf2` does, and fails loudly if it is missing.
"""
