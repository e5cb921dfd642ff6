"""MI355X-native GMRF posterior-precision solves (PCG mean, perturbation sample,
Hutchinson trace) for the spatial GLM of Siden, Eklund, Bolin and Villani.

The compute path lives in the HIP library ``libgmrf.so`` built from ``csrc/``;
``paper_1606_00980_amd.gmrf`` is its thin ctypes binding.  ``synth`` generates
seeded synthetic workloads.
"""
__all__ = ["gmrf", "synth"]
