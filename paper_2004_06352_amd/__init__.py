"""MI355X-native lens-gradient library (Lenstool-HPC hot path, arXiv:2004.06352).

Importing the package loads nothing native.  The HIP library and its Python
binding load on first use of a binding name (``grad_map``, ``hessian_map``,
``chi2_batch``, ...) and raise if the built library is missing.
"""
import importlib

_SUBMODULES = {"inputs", "binding", "build", "serve", "tune", "batch"}


def __getattr__(name):
    if name in _SUBMODULES or name.startswith("_"):
        raise AttributeError(name)
    binding = importlib.import_module(__name__ + ".binding")
    try:
        return getattr(binding, name)
    except AttributeError:
        raise AttributeError(name) from None
