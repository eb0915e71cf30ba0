"""MI355X-native FAS multigrid with weighted overlapping Schwarz smoothing for SIPG DG-SEM.

The compute path is the HIP library ``libdgfas.so`` (C ABI in include/dgfas.h);
``binding`` wraps it with ctypes.  ``workloads`` builds seeded synthetic meshes.
"""
__all__ = ['binding', 'workloads']
