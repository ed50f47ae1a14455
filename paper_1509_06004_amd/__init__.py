"""Exact parametric max-flow / min s-t cut on image grids, MI355X-native.

The compute path is the HIP library ``libpmf.so`` (C ABI declared in
``include/pmf.h``); :mod:`paper_1509_06004_amd.pmf` is its Python binding and
:mod:`paper_1509_06004_amd.workload` produces the seeded synthetic instances.
Nothing is imported eagerly so that the generator can be used without a GPU.
"""

__all__ = ["workload", "pmf"]
