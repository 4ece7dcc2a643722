"""MI355X-native Vertex Block Descent (VBD) hot path.

The solver lives in a HIP/C++ shared library with a C ABI (include/vbd.h);
this package is its thin Python binding.  ``workloads`` holds the seeded
synthetic input generators.  The binding is imported lazily so that the
generators can be used without the native library.
"""
__all__ = ["Topology", "Rollout", "probe_copy", "StepParams", "workloads"]


def __getattr__(name):
    if name in ("Topology", "Rollout", "probe_copy", "params_struct"):
        from . import api
        return getattr(api, name)
    if name == "StepParams":
        from .workloads import StepParams
        return StepParams
    raise AttributeError(name)
