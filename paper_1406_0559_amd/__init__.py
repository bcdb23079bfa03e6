"""MI355X-native direct inverse ray-shooting (Vernardos & Fluke 2014, Section 2.1).

The compute path is a HIP library for gfx950 behind a C-ABI (include/raylens.h);
`paper_1406_0559_amd.raylens` is its thin ctypes binding. Importing the package
loads nothing: the library is opened on first use and a missing build is an
error, never a fallback.
"""
__all__ = ["inputs", "raylens"]
