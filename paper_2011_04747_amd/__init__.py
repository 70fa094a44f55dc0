"""MI355X-native DAETI monodomain solver (dual adaptive explicit time integration).

The solver lives in the HIP library ``libmono.so`` behind the C interface of
``include/mono.h``; :mod:`paper_2011_04747_amd.mono` is its thin ctypes
binding and :mod:`paper_2011_04747_amd.workloads` describes the synthetic
problems.  Importing the package loads neither.
"""
__all__ = ["mono", "workloads"]
