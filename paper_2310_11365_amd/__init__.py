"""MI355X-native fine propagator and MC-moments Parareal driver (arXiv 2310.11365).

The compute path is the HIP library ``libmcpr.so`` (C ABI declared in
``include/mcpr.h``); :mod:`paper_2310_11365_amd.mcpr` is its ctypes binding.
Importing this package loads nothing; the binding loads the library on first
use and raises if it is missing.
"""
__all__ = ["mcpr", "workloads"]
