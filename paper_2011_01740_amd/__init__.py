"""MI355X-native ensemble integrator for many independent low-dimensional ODEs.

The compute path is the HIP library ``libens.so`` (C ABI declared in
``include/ens.h``); :mod:`paper_2011_01740_amd.ens` is its thin Python binding.
Importing this package loads nothing; the binding loads the library on first
use and raises if it is missing.
"""
__all__ = ["inputs"]
