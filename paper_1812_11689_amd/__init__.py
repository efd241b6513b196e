"""rpForests kNN search on AMD MI355X (gfx950): HIP kernels behind a C ABI.

The compute path lives in the shared library built from `csrc/` (see `_lib.py` for the
ctypes binding).  `workloads` holds the seeded synthetic input generators.
"""
