"""sorlayout: SOR-accelerated stress-majorization graph layout on MI355X.

The compute path is a C-ABI HIP library (``libsorlayout.so``, declared in
``include/sorlayout.h``); ``paper_1711_01228_amd.binding`` marshals arguments
to it.  ``paper_1711_01228_amd.inputs`` draws seeded synthetic graphs and
starting placements.  Importing this package loads neither torch nor the
library; ``binding`` does, and raises if the library is missing.
"""
__all__ = ["inputs", "binding"]


def __getattr__(name):
    if name in ("binding", "inputs"):
        import importlib

        return importlib.import_module(__name__ + "." + name)
    raise AttributeError(name)
