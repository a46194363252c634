"""MI355X-native free-energy lattice Boltzmann (FRE LBM) step.

The hot path is the HIP library ``libfrelbm.so`` (C ABI: include/frelbm.h),
built with ``python -m paper_2212_01617_amd.build``; ``frelbm`` is its ctypes
binding, ``synth`` builds seeded synthetic inputs.
"""
__all__ = ["frelbm", "synth"]
