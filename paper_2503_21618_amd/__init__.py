"""SLRF eigensolver for gfx950: the binding (``binding``) is loaded on first use.

``import paper_2503_21618_amd.build`` does not touch the compiled library; any
other attribute (Solver, design_poles, ...) loads libslrf.so and raises if it
has not been built.
"""
import importlib


def __getattr__(name):
    if name.startswith("__"):
        raise AttributeError(name)
    mod = importlib.import_module(__name__ + ".binding")
    return mod if name == "binding" else getattr(mod, name)
