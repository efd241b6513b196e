"""rpForests kNN search on AMD MI355X (gfx950): HIP kernels behind a C ABI.

`rpf` is the ctypes binding of the library built from `csrc/` (`build.py`);
`workloads` holds the seeded synthetic input generators.  Attributes of `rpf`
(build, depth, Forest, ...) are also reachable from the package itself.
"""

import importlib


def __getattr__(name):
    if name in ("rpf", "workloads", "build"):  # submodules (`build` compiles the library)
        return importlib.import_module(f"{__name__}.{name}")
    mod = importlib.import_module(f"{__name__}.rpf")
    return getattr(mod, name)
