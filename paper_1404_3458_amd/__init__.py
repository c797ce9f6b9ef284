"""MI355X-native novel-polynomial-basis Reed-Solomon erasure codec.

The compute path lives in the HIP library ``librs_nb.so`` (built from
``csrc/``); :mod:`paper_1404_3458_amd.rs` is a thin ctypes binding over its
C ABI (``include/rs.h``).  :mod:`paper_1404_3458_amd.synth` holds the seeded
synthetic input generators.
"""
