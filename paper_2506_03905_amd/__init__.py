"""MI355X (gfx950) implementation of the LBM-RANS hot path of Ponsin & Lozano,
"Lattice Boltzmann wall boundary conditions for RANS-based simulations with
wall functions" (arXiv 2506.03905).

The arithmetic lives in the HIP library ``liblbm.so`` (C ABI in
``include/lbm.h``); :mod:`paper_2506_03905_amd.lbm` is a thin ctypes binding
with the same names, :mod:`.units` the host-side unit conversion and
:mod:`.inputs` the seeded synthetic workloads.  Importing the package does not
load the library; the first call into :mod:`.lbm` does, and fails loudly if it
is missing.
"""
