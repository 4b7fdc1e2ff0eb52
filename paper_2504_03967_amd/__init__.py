"""MI355X-native state-vector circuit simulator (Q-GEAR hot path, arXiv 2504.03967).

Submodules are imported lazily so that the workload generators can be used
without a GPU runtime:
  * ``workloads`` -- seeded circuit generators (no simulation arithmetic);
  * ``qg``        -- ctypes binding of the C-ABI library ``libqg.so``.
"""
import importlib

__all__ = ["workloads", "qg"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
