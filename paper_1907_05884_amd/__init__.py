"""MI355X (gfx950) randomized functional sparse Tucker: Python binding of libfst.

Attribute access is forwarded to ``paper_1907_05884_amd.binding``, which loads libfst.so on
first use and raises ImportError if it has not been built
(``python -m paper_1907_05884_amd.build``).  Keeping the load lazy lets the build script run
from this package without a library present.
"""
import importlib as _importlib


def __getattr__(name):
    if name.startswith("__") or name in ("binding", "build"):
        raise AttributeError(name)
    return getattr(_importlib.import_module(__name__ + ".binding"), name)
