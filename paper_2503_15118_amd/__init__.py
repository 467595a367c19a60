"""sparqs: the sparse register-level simulator hot path on one AMD MI355X.

``State`` (and the rest of the C-ABI binding) lives in ``_abi``; importing it
loads ``libsparqs.so`` and raises if the library has not been built.
"""

__all__ = ["State", "state_for_circuit", "SSError"]


def __getattr__(name):
    if name in __all__:
        from . import _abi
        return getattr(_abi, name)
    raise AttributeError(name)
