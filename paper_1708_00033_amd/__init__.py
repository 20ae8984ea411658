"""MI355X-native direct closed-shell Hartree-Fock Fock build.

The compute path is the HIP library ``libhfx.so`` (C ABI in include/hfx.h);
``paper_1708_00033_amd.hfx`` is its ctypes binding.  The binding is loaded
lazily so that ``paper_1708_00033_amd.build`` can run before the library
exists.
"""
import importlib

__all__ = ["hfx", "build"]


def __getattr__(name):
    if name in ("hfx", "build"):
        return importlib.import_module(f"{__name__}.{name}")
    if name == "Context":
        return importlib.import_module(f"{__name__}.hfx").Context
    raise AttributeError(name)
