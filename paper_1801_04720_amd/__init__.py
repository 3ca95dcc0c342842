"""MI355X (gfx950) hot path of "Combining Stereo Disparity and Optical Flow for
Basic Scene Flow" (arXiv 1801.04720): SGM stereo at two time steps and the
combination into sparse scene flow, as hand-written HIP kernels behind the C
ABI in include/sf.h.  This package holds the Python binding, the build step
and the seeded synthetic workloads; `import paper_1801_04720_amd` does not
touch the GPU.
"""
from __future__ import annotations

__all__ = ["api", "synth", "build_lib", "lib_path"]


def build_lib() -> str:
    from .build import build

    return build()


def lib_path() -> str:
    from ._lib import LIB_PATH

    return LIB_PATH


def __getattr__(name):
    if name in ("api", "pipeline", "lrnet", "batch"):
        import importlib

        return importlib.import_module("." + name, __name__)
    raise AttributeError(name)
