"""MI355X-native full-batch SPFOM for the GAM choice-based LP.

``instances`` draws seeded synthetic inputs; ``cblp`` binds the HIP library
``libcblp.so`` (built from ``csrc/``), whose C ABI is ``include/cblp.h``.
The binding is imported lazily so that the input generator works on hosts
without torch's HIP runtime.
"""

__all__ = ["instances", "cblp"]


def __getattr__(name):
    if name in __all__:
        import importlib
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
