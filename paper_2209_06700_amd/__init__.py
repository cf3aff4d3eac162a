"""MI355X-native stage-parallel Radau IIA solver for the FE heat equation.

The compute path is the HIP library ``librk.so`` (C ABI: include/rk.h); the
Python module ``rk`` is its binding.  ``build`` compiles the library.
"""
