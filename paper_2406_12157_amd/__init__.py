"""MI355X-native finite-volume stochastic heat / Dean-Kawasaki solver.

The compute path is the HIP library ``libshe.so`` (C ABI in ``include/she.h``);
``paper_2406_12157_amd.she`` is its ctypes binding and
``paper_2406_12157_amd.workloads`` holds the seeded synthetic workloads.
Submodules are imported lazily so that the workload generators do not need
the built library.
"""
__all__ = ["she", "workloads", "build"]
