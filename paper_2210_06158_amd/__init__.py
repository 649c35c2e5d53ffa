"""Hybrid depth-of-field pass for MI355X (gfx950).

The pass itself lives in the HIP library ``libdof.so`` behind a C ABI
(``include/dof.h``); :mod:`paper_2210_06158_amd.dof` is its thin ctypes binding
and :mod:`paper_2210_06158_amd.synth` generates seeded synthetic inputs.
Importing this package does not load the GPU library.
"""
