"""MI355X (gfx950) Local Directional Pattern extraction.

The HIP kernels and their C ABI live in ``libldp.so`` (built from ``csrc/``);
``binding`` wraps them for torch device tensors.  ``synth`` generates the
seeded synthetic inputs.  Importing the package does not load the library;
the first call does, and raises if it has not been built.
"""
__all__ = ["binding", "synth", "build"]


def __getattr__(name):
    if name in ("codes", "histograms", "extract", "BatchPlan", "LdpError", "Server"):
        from . import binding
        return getattr(binding, name)
    raise AttributeError(name)
