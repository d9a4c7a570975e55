"""MI355X-native FP64 Lindblad master-equation evolution (gfx950 HIP kernels).

The library proper is the C-ABI shared object ``liblme.so`` built from
``csrc/``; :mod:`paper_1110_0573_amd.lme` is its thin ctypes binding and
:mod:`paper_1110_0573_amd.systems` builds seeded example systems.
"""
