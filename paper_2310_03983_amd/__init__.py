"""MI355X-native min-plus all-pairs shortest paths (arXiv 2310.03983).

The compute path is libapsp.so (hand-written HIP for gfx950) behind the C ABI
in include/apsp.h.  ``paper_2310_03983_amd.apsp`` is its Python binding;
``paper_2310_03983_amd.graphgen`` is the seeded synthetic graph generator.
The binding is imported lazily so that the generator works without the
native library.
"""
__all__ = ["apsp", "graphgen"]


def __getattr__(name):
    if name in ("apsp", "graphgen"):
        import importlib
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
