"""libpsdproj: PSD-cone projection by composite polynomial filtering on MI355X.

The HIP library (``libpsdproj.so``, built from ``csrc/``) does all the work;
``psdproj`` is its ctypes binding and ``inputs`` draws seeded synthetic
workloads. Submodules are imported on demand so that the input generators can
be used without the library.
"""
__all__ = ["psdproj", "inputs"]
