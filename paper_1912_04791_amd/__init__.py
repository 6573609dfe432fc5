"""MI355X-native A-DOT hot path: HIP kernels for gfx950 behind a small C ABI.

``paper_1912_04791_amd.dsve`` is the ctypes binding to ``libdsve.so`` (the only
compute path; it raises if the library is missing).  ``inputs`` builds seeded
synthetic workloads and holds none of the scheme's arithmetic.
"""
__all__ = ["dsve", "inputs"]


def __getattr__(name):
    if name in __all__:
        import importlib
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
