"""MI355X (gfx950) sliced tensor-network contraction of random-quantum-circuit
amplitudes.

``paper_2111_01066_amd.tnrcs`` is the ctypes binding of ``libtnrcs.so`` (C ABI in
``include/tnrcs.h``); ``paper_2111_01066_amd.build`` compiles the library with
hipcc for gfx950.  The binding is imported lazily so that the build step can
run before the library exists.
"""
import importlib

__all__ = ["tnrcs", "build"]


def __getattr__(name):
    if name in ("tnrcs", "build"):
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
