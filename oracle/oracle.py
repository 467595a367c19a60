"""Python driver for the CPU oracle (test infrastructure only).

Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg use this
module.  It marshals a neutral op list (``workloads.OP_DTYPE``) into the
oracle's own record layout and calls ``liboracle.so`` (built from
``sparse_oracle.cpp`` with ``-O2 -ffp-contract=off``).  Nothing here, or in the
library, is shared with the HIP path.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Tuple

import numpy as np

import workloads as wl

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sparse_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

ORA_OP = np.dtype([
    ("kind", "u4"), ("nctl", "u4"), ("reg", "u4"), ("reg2", "u4"), ("table", "u4"), ("reg3", "u4"),
    ("qmask", "u8"), ("imm", "u8"), ("theta", "f8"),
    ("ctl_reg", "u4", (3,)), ("ctl_qubit", "u4", (3,)), ("ctl_val", "u4", (3,)), ("reg4", "u4"),
])
assert ORA_OP.itemsize == 88  # matches struct ora_op

# oracle kind codes (its own enumeration) by op name
_ORA_KIND = {"X": 0, "H": 1, "RY": 2, "ADD": 3, "SUB": 4, "MULC": 5, "XOR": 6, "XORC": 7,
             "QRAM_LOAD": 8, "QRAM_UNLOAD": 9, "REFLECT0": 10,
             "Y": 11, "Z": 12, "S": 13, "SDG": 14, "T": 15, "TDG": 16, "PHASE": 17, "ROT": 18,
             "ADDC": 19, "MUL": 20, "DIV": 21}


def build(force: bool = False) -> str:
    """Compile the oracle library with g++ (plain C++17, no fused multiply-add)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
               "-shared", "-o", _LIB + ".tmp", _SRC]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = ctypes.CDLL(build())
        vp, u32, u64, f64 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double
        P = ctypes.POINTER
        L.ora_create.restype = vp
        L.ora_create.argtypes = [P(u32), u32, f64]
        L.ora_destroy.argtypes = [vp]
        L.ora_layout.argtypes = [vp, u32, P(u32), P(u32)]
        L.ora_add_table.argtypes = [vp, P(u64), u64, u32, u32]
        L.ora_add_matrix.argtypes = [vp, P(f64)]
        L.ora_add_register.argtypes = [vp, u32]
        L.ora_remove_register.argtypes = [vp, u32]
        L.ora_probabilities.restype = u64
        L.ora_probabilities.argtypes = [vp, u32, P(u64), P(f64), u64]
        L.ora_set_entries.argtypes = [vp, P(u64), P(f64), u64]
        L.ora_apply.argtypes = [vp, vp, u64, P(f64), P(u64)]
        L.ora_prune.argtypes = [vp, f64]
        L.ora_measure.argtypes = [vp, u32, f64, P(u64), P(f64)]
        L.ora_nnz.restype = u64
        L.ora_nnz.argtypes = [vp]
        L.ora_peak.restype = u64
        L.ora_peak.argtypes = [vp]
        L.ora_export.restype = u64
        L.ora_export.argtypes = [vp, P(u64), P(u64), P(f64), u64]
        _lib = L
    return _lib


def _ptr(a, t):
    return a.ctypes.data_as(ctypes.POINTER(t))


def to_oracle_ops(ops: np.ndarray) -> np.ndarray:
    out = np.zeros(len(ops), dtype=ORA_OP)
    names = [wl.KINDS[int(k)] for k in ops["kind"]]
    out["kind"] = [_ORA_KIND[n] for n in names]
    for f in ("nctl", "reg", "reg2", "reg3", "reg4", "table", "qmask", "imm", "theta"):
        out[f] = ops[f]
    out["ctl_reg"] = ops["ctl_reg"]
    out["ctl_qubit"] = ops["ctl_qubit"]
    out["ctl_val"] = ops["ctl_val"]
    return out


class OracleState:
    """One oracle instance: a std::map from packed key to complex amplitude."""

    def __init__(self, regs, eps: float = 1e-14, tables=(), init_values=None, init_amps=None, matrices=()):
        L = lib()
        self.nregs = len(regs)
        widths = np.array([w for _, w in regs], dtype=np.uint32)
        self.h = L.ora_create(_ptr(widths, ctypes.c_uint32), len(widths), float(eps))
        if not self.h:
            raise ValueError("oracle: bad register layout")
        for t in tables:
            v = np.ascontiguousarray(t.values, dtype=np.uint64)
            rc = L.ora_add_table(self.h, _ptr(v, ctypes.c_uint64), len(v), t.addr_bits, t.word_bits)
            if rc < 0:
                raise ValueError("oracle: bad table")
        for m in matrices:
            m8 = np.ascontiguousarray(np.asarray(m, dtype=np.complex128).reshape(2, 2)).view(np.float64).ravel()
            L.ora_add_matrix(self.h, _ptr(m8, ctypes.c_double))
        if init_values is not None:
            self.set_entries(init_values, init_amps)

    @classmethod
    def from_circuit(cls, c: "wl.Circuit") -> "OracleState":
        return cls(c.regs, c.eps, c.tables, c.init_values, c.init_amps, c.matrices)

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            lib().ora_destroy(h)
            self.h = None

    def set_entries(self, values, amps):
        v = np.ascontiguousarray(values, dtype=np.uint64).reshape(-1, self.nregs)
        a = np.ascontiguousarray(np.asarray(amps, dtype=np.complex128)).view(np.float64)
        if lib().ora_set_entries(self.h, _ptr(v, ctypes.c_uint64), _ptr(a, ctypes.c_double), len(v)):
            raise ValueError("oracle: duplicate keys")

    def apply(self, ops: np.ndarray) -> Tuple[float, int]:
        rec = to_oracle_ops(ops)
        sec = ctypes.c_double(0.0)
        ein = ctypes.c_uint64(0)
        rc = lib().ora_apply(self.h, rec.ctypes.data_as(ctypes.c_void_p), len(rec),
                             ctypes.byref(sec), ctypes.byref(ein))
        if rc:
            raise RuntimeError(f"oracle: apply failed ({rc})")
        return sec.value, ein.value

    def prune(self, eps: float):
        lib().ora_prune(self.h, float(eps))

    def measure(self, reg: int, u: float) -> Tuple[int, float]:
        out = ctypes.c_uint64(0)
        p = ctypes.c_double(0.0)
        if lib().ora_measure(self.h, reg, float(u), ctypes.byref(out), ctypes.byref(p)):
            raise RuntimeError("oracle: measure failed")
        return out.value, p.value

    def add_register(self, width: int) -> int:
        r = lib().ora_add_register(self.h, int(width))
        if r < 0:
            raise ValueError("oracle: no room for the register")
        self.nregs += 1
        return r

    def remove_register(self, reg: int):
        if lib().ora_remove_register(self.h, int(reg)):
            raise ValueError("oracle: the register does not hold one value in every branch")

    def probabilities(self, reg: int):
        """(values, p(v)/P) ascending, without collapse."""
        n = int(lib().ora_probabilities(self.h, reg, None, None, 0))
        v = np.zeros(n, dtype=np.uint64)
        p = np.zeros(n, dtype=np.float64)
        lib().ora_probabilities(self.h, reg, _ptr(v, ctypes.c_uint64), _ptr(p, ctypes.c_double), n)
        return v, p

    def layout(self, reg: int) -> Tuple[int, int]:
        w = ctypes.c_uint32(0)
        o = ctypes.c_uint32(0)
        lib().ora_layout(self.h, reg, ctypes.byref(w), ctypes.byref(o))
        return w.value, o.value

    @property
    def nnz(self) -> int:
        return int(lib().ora_nnz(self.h))

    @property
    def peak(self) -> int:
        return int(lib().ora_peak(self.h))

    def export(self):
        """(keys[n,4] uint64, values[n,nregs] uint64, amps[n] complex128), ascending key."""
        n = self.nnz
        keys = np.zeros((n, 4), dtype=np.uint64)
        vals = np.zeros((n, max(self.nregs, 1)), dtype=np.uint64)
        amps = np.zeros(n, dtype=np.complex128)
        got = lib().ora_export(self.h, _ptr(keys, ctypes.c_uint64), _ptr(vals, ctypes.c_uint64),
                               _ptr(amps.view(np.float64), ctypes.c_double), n)
        assert got == n
        return keys, vals[:, :self.nregs], amps


def run_circuit(c: "wl.Circuit", ops: Optional[np.ndarray] = None):
    """Run a whole circuit; returns (OracleState, seconds, entries_in)."""
    st = OracleState.from_circuit(c)
    sec, ein = st.apply(c.ops if ops is None else ops)
    return st, sec, ein
