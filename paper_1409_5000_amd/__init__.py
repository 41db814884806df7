"""MI355X-native Estrada-Benzi total-communicability engine (Krylov exp(A) 1 over graph realizations).

The compute path is the HIP library libebtc.so (C ABI in include/ebtc.h); `api` is its torch-facing
binding. Nothing here falls back to a CPU implementation.
"""
import importlib

from . import _abi  # noqa: F401

__all__ = ["_abi", "api"]


def __getattr__(name):
    if name == "api":
        return importlib.import_module(".api", __name__)
    raise AttributeError(name)
