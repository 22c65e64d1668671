"""MI355X-native batched skip-list index (PI, arXiv 1601.00159).

The hot path lives in libpi.so (HIP kernels for gfx950, C ABI in
include/pi.h); this package only marshals arguments to it.

    from paper_1601_00159_amd import Index
    ix = Index()
    ix.bulk_load(keys, values)
    out_values, out_status = ix.execute(ops, keys, values)
"""
__all__ = ["Index", "workloads"]


def __getattr__(name):
    if name == "Index":
        from .index import Index
        return Index
    raise AttributeError(name)
