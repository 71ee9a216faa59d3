"""MI355X-native differentiable Gaussian rasterizer and AdpSplit adaptive split.

Every step of the path runs in the HIP kernels of ``libadpsplit.so`` (built
from ``csrc/``) behind the C-ABI declared in ``include/adpsplit.h``; the
Python modules only marshal arguments.  Importing the package does not load
the library; the first call into ``api`` does, and raises if it is missing.
"""
__version__ = "0.1.0"


def __getattr__(name):
    if name in ("api", "synth", "autograd", "autotune", "serve", "train", "sweep", "densify"):
        import importlib
        return importlib.import_module("." + name, __name__)
    raise AttributeError(name)
