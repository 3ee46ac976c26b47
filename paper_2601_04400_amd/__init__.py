"""MI355X-native WENO5 / HLLC / immersed-boundary / SSP-RK3 hot path of
arXiv 2601.04400, behind the C ABI of include/shk.h (libshk.so).

Submodules:
  solver  -- Grid: torch-owned memory and streams around the C ABI
  inputs  -- seeded synthetic initial data and level sets (no solver arithmetic)
  build   -- hipcc build of libshk.so for gfx950
"""
import importlib

__all__ = ["Grid", "normal_shock_state", "inputs", "solver"]


def __getattr__(name):
    if name in ("Grid", "normal_shock_state"):
        return getattr(importlib.import_module(".solver", __name__), name)
    if name in ("inputs", "solver", "build"):
        return importlib.import_module("." + name, __name__)
    raise AttributeError(name)
