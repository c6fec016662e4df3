"""MI355X-native HISQ even/odd Dslash and CG solvers (HIP for gfx950).

The compute library is ``libhisq.so`` (C ABI in ``include/hisq.h``); the
Python binding lives in ``paper_2111_10354_amd.hisq`` and is imported on
first use so that building the library does not require it to exist yet.
"""

__all__ = ["hisq"]


def __getattr__(name):
    if name == "hisq":
        import importlib
        return importlib.import_module(__name__ + ".hisq")
    raise AttributeError(name)
