"""MI355X-native Riemann-SPH multiphase surface-tension hot path.

The compute path is the HIP library ``librsph.so`` (C-ABI declared in
``include/rsph.h``); ``paper_2503_16082_amd.rsph`` is its thin ctypes binding.
``paper_2503_16082_amd.workloads`` builds seeded synthetic inputs.
Importing this package loads nothing; the binding loads the library on first use
and raises if it is not built.
"""
__all__ = ["rsph", "workloads"]
