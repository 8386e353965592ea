"""MI355X (gfx950) implementation of the RPA polarization P(q, i w) and the
screened interaction W of all-electron GW (Friedrich, Bluegel, Schindlmayr).

The compute lives in libgw.so (HIP kernels behind a C ABI, include/gw.h);
``paper_1003_0316_amd.binding`` is its thin Python binding.  Importing an API
name from this package loads the library and fails loudly if it is missing.
"""
import importlib

__all__ = ["binding", "build"]


def __getattr__(name):
    if name.startswith("__"):
        raise AttributeError(name)
    if name in ("build", "surrogate", "train_surrogate"):
        # submodules; the build step must work before the library exists
        return importlib.import_module(__name__ + "." + name)
    b = importlib.import_module(__name__ + ".binding")
    if name == "binding":
        return b
    if hasattr(b, name):
        return getattr(b, name)
    raise AttributeError(name)
