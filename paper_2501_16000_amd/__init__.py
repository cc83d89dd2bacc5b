"""MI355X (gfx950) implementation of the Onsager-regularized lattice Boltzmann
sweep on the D2Q9 lattice, and its D3Q27 extension (arXiv 2501.16000).

Submodules:
  ``oreg``       ctypes binding of ``liboreg.so`` (the C ABI of include/oreg.h);
  ``oreg3``      the D3Q27 entry points (include/oreg3.h);
  ``serve``      continuous-batching serving of many independent lattices;
  ``workloads``  seeded synthetic initial fields and request streams;
  ``build``      in-tree hipcc build of ``liboreg.so``.

``oreg`` is imported on first use so that ``workloads`` stays importable on a
machine where the library has not been built yet.
"""
import importlib

__all__ = ["oreg", "oreg3", "workloads", "build", "serve"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
