"""ctypes binding of ``libsparqs.so`` (the C ABI in include/sparqs.h).

Argument marshalling only: every step of the simulation runs in the HIP
kernels behind the ABI.  PyTorch supplies the device arena (a uint8 CUDA
tensor) and the stream.  If the library has not been built this module raises
at import time; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence, Tuple

import numpy as np

import workloads as wl

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsparqs.so")

SS_OK, SS_E_ARG, SS_E_NOT_UNITARY, SS_E_QRAM, SS_E_CAPACITY, SS_E_NOMEM, SS_E_HIP, SS_E_STATE, SS_E_PLAN = \
    0, -1, -2, -3, -4, -5, -6, -7, -8

# enum ss_kind of include/sparqs.h
SS_KIND = {"X": 0, "H": 1, "RY": 2, "ADD": 3, "SUB": 4, "MULC": 5, "XOR": 6, "XORC": 7,
           "QRAM_LOAD": 8, "QRAM_UNLOAD": 9, "REFLECT0": 10,
           "Y": 11, "Z": 12, "S": 13, "SDG": 14, "T": 15, "TDG": 16, "PHASE": 17, "ROT": 18,
           "ADDC": 19, "MUL": 20, "DIV": 21}

SS_OP = np.dtype([
    ("kind", "<u2"), ("nctl", "u1"), ("flags", "u1"),
    ("reg", "<u4"), ("reg2", "<u4"), ("aux", "<u4"),
    ("qmask", "<u8"), ("imm", "<u8"), ("theta", "<f8"),
    ("ctl", [("reg", "<u4"), ("qubit", "<u2"), ("value", "<u2")], (3,)),
])
assert SS_OP.itemsize == 64


class SSError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = code
        super().__init__(f"{what}: {strerror(code)} ({code})")


class _Reg(ctypes.Structure):
    _fields_ = [("nqubits", ctypes.c_uint32), ("name", ctypes.c_char_p)]


class _Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("failed_inst", ctypes.c_uint32),
                ("failed_op", ctypes.c_uint64), ("nnz", ctypes.c_uint64), ("peak", ctypes.c_uint64)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"HIP library {LIB_PATH} is not built; run __graft_entry__.build() "
                          "(hipcc --offload-arch=gfx950)")
    # The library shares the HIP runtime, the device memory and the streams of
    # PyTorch.  PyTorch ships its own HIP runtime under the same soname, so it
    # is loaded first: the library then binds to that copy instead of bringing
    # in a second runtime that PyTorch would pick up in turn.
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    vp, u32, u64, f64, i32, i64 = (ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double,
                                   ctypes.c_int, ctypes.c_int64)
    P = ctypes.POINTER
    sig = {
        "ss_required_bytes": [P(_Reg), u32, u32, u64, u64, P(ctypes.c_size_t)],
        "ss_create_state": [P(_Reg), u32, u32, f64, vp, ctypes.c_size_t, u64, vp, P(vp)],
        "ss_create_state_noalloc": [P(_Reg), u32, u32, f64, vp, ctypes.c_size_t, u64, vp, P(vp)],
        "ss_destroy_state": [vp],
        "ss_capacity": [vp, P(u64)],
        "ss_layout": [vp, u32, P(u32), P(u32), P(u32)],
        "ss_key_words": [vp, P(u32)],
        "ss_load_qram": [vp, P(u64), u64, u32, u32, P(u32)],
        "ss_load_matrix": [vp, P(f64), P(u32)],
        "ss_set_entries": [vp, u32, P(u64), P(f64), u64],
        "ss_apply_ops": [vp, vp, u64, P(u64), P(_Result)],
        "ss_prune": [vp, f64],
        "ss_measure": [vp, u32, u32, f64, P(u64), P(f64)],
        "ss_probabilities": [vp, u32, u32, P(u64), P(f64), u64, P(u64)],
        "ss_add_register": [vp, u32, ctypes.c_char_p, P(u32)],
        "ss_remove_register": [vp, u32],
        "ss_nnz": [vp, u32, P(u64), P(u64)],
        "ss_export": [vp, u32, P(u64), P(f64), u64, P(u64)],
        "ss_sync": [vp, P(_Result)],
        "ss_rebind_arena": [vp, vp, ctypes.c_size_t],
        "ss_set_option": [vp, ctypes.c_char_p, i64],
        "ss_stats": [vp, P(u64)],
        "ss_trace_read": [vp, u32, P(u64), P(f64), P(u64), P(u64)],
        "ss_device_error": [vp, P(u32)],
        "ss_graph_capture": [vp, vp, u64, P(u64), P(_Result), P(vp)],
        "ss_graph_launch": [vp, P(_Result)],
        "ss_graph_destroy": [vp],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = i32
    L.ss_strerror.argtypes = [i32]
    L.ss_strerror.restype = ctypes.c_char_p
    return L


lib = _load()

EXPORTED = ("ss_required_bytes", "ss_create_state", "ss_create_state_noalloc", "ss_destroy_state", "ss_capacity", "ss_layout",
            "ss_key_words", "ss_load_qram", "ss_load_matrix", "ss_set_entries", "ss_apply_ops", "ss_prune", "ss_measure",
            "ss_probabilities", "ss_add_register", "ss_remove_register",
            "ss_nnz", "ss_export", "ss_sync", "ss_rebind_arena", "ss_set_option", "ss_stats",
            "ss_trace_read", "ss_device_error", "ss_strerror", "ss_graph_capture", "ss_graph_launch",
            "ss_graph_destroy")

TRACE_CATS = ("perm", "sort_hist", "sort_pass", "group", "expand", "filter")


def strerror(code: int) -> str:
    return lib.ss_strerror(code).decode()


def _check(rc: int, what: str):
    if rc != SS_OK:
        raise SSError(rc, what)


def _p(a, t):
    return a.ctypes.data_as(ctypes.POINTER(t))


def to_ss_ops(ops: np.ndarray) -> np.ndarray:
    """Neutral op records (workloads.OP_DTYPE) -> ss_op records."""
    out = np.zeros(len(ops), dtype=SS_OP)
    if len(ops) == 0:
        return out
    names = [wl.KINDS[int(k)] for k in ops["kind"]]
    out["kind"] = [SS_KIND[n] for n in names]
    out["nctl"] = ops["nctl"]
    out["reg"] = ops["reg"]
    out["reg2"] = ops["reg2"]
    # aux: the QRAM table or ROT matrix index, or MUL / DIV's third register;
    # DIV's remainder register travels in imm
    kinds = np.array(names)
    third = (kinds == "MUL") | (kinds == "DIV")
    out["aux"] = np.where(third, ops["reg3"], ops["table"])
    out["qmask"] = ops["qmask"]
    out["imm"] = np.where(kinds == "DIV", ops["reg4"].astype(np.uint64), ops["imm"])
    out["theta"] = ops["theta"]
    out["ctl"]["reg"] = ops["ctl_reg"]
    out["ctl"]["qubit"] = ops["ctl_qubit"]
    out["ctl"]["value"] = ops["ctl_val"]
    return out


def _regs(regs: Sequence[Tuple[str, int]]):
    arr = (_Reg * len(regs))()
    for i, (name, w) in enumerate(regs):
        arr[i].nqubits = int(w)
        arr[i].name = None
    return arr


def required_bytes(regs, ninst: int, cap_entries: int, table_bytes: int = 0) -> int:
    b = ctypes.c_size_t(0)
    _check(lib.ss_required_bytes(_regs(regs), len(regs), ninst, cap_entries, table_bytes, ctypes.byref(b)),
           "ss_required_bytes")
    return int(b.value)


class State:
    """A sparse state on one GPU, held in a caller-owned torch arena."""

    def __init__(self, regs, ninst: int = 1, eps: float = 1e-14, cap_entries: int = 1 << 16,
                 table_bytes: int = 1 << 20, device=None, stream=None, arena_bytes: Optional[int] = None,
                 noalloc: bool = False):
        """noalloc: create through ss_create_state_noalloc (scratch in the
        library's own device array; the torch buffer holds tables and entries
        only, sized here like a full arena)."""
        import torch
        self.torch = torch
        self.regs = list(regs)
        self.ninst = ninst
        self.eps = eps
        self.device = torch.device(device if device is not None else "cuda:0")
        if arena_bytes is None:
            arena_bytes = required_bytes(self.regs, ninst, cap_entries, table_bytes)
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p(0)
        create = lib.ss_create_state_noalloc if noalloc else lib.ss_create_state
        _check(create(_regs(self.regs), len(self.regs), ninst, float(eps),
                      ctypes.c_void_p(self.arena.data_ptr()), int(arena_bytes), int(table_bytes),
                      ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)),
               "ss_create_state_noalloc" if noalloc else "ss_create_state")
        self.h = h
        self.table_ids = []
        self.table_bytes = int(table_bytes)

    def rebind(self, cap_entries: int):
        """Move the state into a new arena sized for `cap_entries` entries."""
        nb = required_bytes(self.regs, self.ninst, cap_entries, self.table_bytes)
        arena = self.torch.empty(int(nb), dtype=self.torch.uint8, device=self.device)
        _check(lib.ss_rebind_arena(self.h, ctypes.c_void_p(arena.data_ptr()), int(nb)), "ss_rebind_arena")
        self.arena = arena

    def close(self):
        if getattr(self, "h", None):
            lib.ss_destroy_state(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- layout -------------------------------------------------------------
    @property
    def key_words(self) -> int:
        w = ctypes.c_uint32(0)
        _check(lib.ss_key_words(self.h, ctypes.byref(w)), "ss_key_words")
        return int(w.value)

    @property
    def capacity(self) -> int:
        c = ctypes.c_uint64(0)
        _check(lib.ss_capacity(self.h, ctypes.byref(c)), "ss_capacity")
        return int(c.value)

    def layout(self, reg: int) -> Tuple[int, int, int]:
        w, o, n = ctypes.c_uint32(0), ctypes.c_uint32(0), ctypes.c_uint32(0)
        _check(lib.ss_layout(self.h, reg, ctypes.byref(w), ctypes.byref(o), ctypes.byref(n)), "ss_layout")
        return int(w.value), int(o.value), int(n.value)

    # -- data ---------------------------------------------------------------
    def load_qram(self, table: "wl.Table") -> int:
        v = np.ascontiguousarray(table.values, dtype=np.uint64)
        qid = ctypes.c_uint32(0)
        _check(lib.ss_load_qram(self.h, _p(v, ctypes.c_uint64), len(v), table.addr_bits, table.word_bits,
                                ctypes.byref(qid)), "ss_load_qram")
        self.table_ids.append(int(qid.value))
        return int(qid.value)

    def load_matrix(self, m) -> int:
        """Register a 2x2 complex matrix (row = output bit) for ROT ops."""
        m8 = np.ascontiguousarray(np.asarray(m, dtype=np.complex128).reshape(2, 2)).view(np.float64).ravel()
        mid = ctypes.c_uint32(0)
        _check(lib.ss_load_matrix(self.h, _p(m8, ctypes.c_double), ctypes.byref(mid)), "ss_load_matrix")
        return int(mid.value)

    def set_entries(self, inst: int, values, amps):
        v = np.ascontiguousarray(values, dtype=np.uint64).reshape(-1, len(self.regs))
        a = np.ascontiguousarray(np.asarray(amps, dtype=np.complex128)).view(np.float64)
        _check(lib.ss_set_entries(self.h, inst, _p(v, ctypes.c_uint64), _p(a, ctypes.c_double), len(v)),
               "ss_set_entries")

    def apply(self, ops: np.ndarray, inst_offsets=None, raise_on_error: bool = True) -> _Result:
        """Apply ops to every instance, or with ``inst_offsets`` (ninst + 1
        CSR offsets into ``ops``) instance i runs ops[off[i]:off[i+1]]."""
        rec = ops if ops.dtype == SS_OP else to_ss_ops(ops)
        rec = np.ascontiguousarray(rec)
        res = _Result()
        offp = None
        if inst_offsets is not None:
            off = np.ascontiguousarray(inst_offsets, dtype=np.uint64)
            if len(off) != self.ninst + 1:
                raise ValueError("inst_offsets needs ninst + 1 entries")
            offp = _p(off, ctypes.c_uint64)
        rc = lib.ss_apply_ops(self.h, ctypes.c_void_p(rec.ctypes.data), len(rec), offp, ctypes.byref(res))
        if rc != SS_OK and raise_on_error:
            bits = ctypes.c_uint32(0)
            lib.ss_device_error(self.h, ctypes.byref(bits))
            raise SSError(rc, f"ss_apply_ops (op {res.failed_op}, device error bits {bits.value})")
        res.status = rc
        return res

    def prune(self, eps: float):
        _check(lib.ss_prune(self.h, float(eps)), "ss_prune")

    def measure(self, inst: int, reg: int, u: float) -> Tuple[int, float]:
        out = ctypes.c_uint64(0)
        p = ctypes.c_double(0.0)
        _check(lib.ss_measure(self.h, inst, reg, float(u), ctypes.byref(out), ctypes.byref(p)), "ss_measure")
        return int(out.value), float(p.value)

    def probabilities(self, inst: int, reg: int):
        """(values, p(v)/P) of register `reg` in instance `inst`, ascending, without collapse."""
        n = ctypes.c_uint64(0)
        _check(lib.ss_probabilities(self.h, inst, reg, None, None, 0, ctypes.byref(n)), "ss_probabilities")
        v = np.zeros(n.value, dtype=np.uint64)
        p = np.zeros(n.value, dtype=np.float64)
        m = ctypes.c_uint64(0)
        _check(lib.ss_probabilities(self.h, inst, reg, _p(v, ctypes.c_uint64), _p(p, ctypes.c_double), len(v),
                                    ctypes.byref(m)), "ss_probabilities")
        assert m.value == len(v)
        return v, p

    def add_register(self, nqubits: int, name: str = "") -> int:
        r = ctypes.c_uint32(0)
        _check(lib.ss_add_register(self.h, int(nqubits), name.encode() or None, ctypes.byref(r)), "ss_add_register")
        self.regs = list(self.regs) + [(name or f"r{r.value}", int(nqubits))]
        return int(r.value)

    def remove_register(self, reg: int):
        _check(lib.ss_remove_register(self.h, int(reg)), "ss_remove_register")

    def nnz(self, inst: int = 0xFFFFFFFF) -> int:
        n = ctypes.c_uint64(0)
        pk = ctypes.c_uint64(0)
        _check(lib.ss_nnz(self.h, inst, ctypes.byref(n), ctypes.byref(pk)), "ss_nnz")
        return int(n.value)

    def peak(self) -> int:
        n = ctypes.c_uint64(0)
        pk = ctypes.c_uint64(0)
        _check(lib.ss_nnz(self.h, 0xFFFFFFFF, ctypes.byref(n), ctypes.byref(pk)), "ss_nnz")
        return int(pk.value)

    def export(self, inst: int = 0):
        """(keys[n, W] uint64, amps[n] complex128) in ascending key order."""
        W = self.key_words
        n = self.nnz(inst) if self.ninst > 1 else self.nnz()
        keys = np.zeros((max(n, 1), W), dtype=np.uint64)
        amps = np.zeros(max(n, 1), dtype=np.complex128)
        got = ctypes.c_uint64(0)
        _check(lib.ss_export(self.h, inst, _p(keys, ctypes.c_uint64), _p(amps.view(np.float64), ctypes.c_double),
                             n, ctypes.byref(got)), "ss_export")
        m = min(int(got.value), n)
        return keys[:m], amps[:m]

    def capture(self, ops: np.ndarray, inst_offsets=None, raise_on_error: bool = True) -> "Graph":
        """Apply ops (as ``apply``) and capture them into a replayable HIP graph."""
        rec = np.ascontiguousarray(ops if ops.dtype == SS_OP else to_ss_ops(ops))
        res = _Result()
        offp = None
        if inst_offsets is not None:
            off = np.ascontiguousarray(inst_offsets, dtype=np.uint64)
            if len(off) != self.ninst + 1:
                raise ValueError("inst_offsets needs ninst + 1 entries")
            offp = _p(off, ctypes.c_uint64)
        g = ctypes.c_void_p(0)
        rc = lib.ss_graph_capture(self.h, ctypes.c_void_p(rec.ctypes.data), len(rec), offp, ctypes.byref(res),
                                  ctypes.byref(g))
        res.status = rc
        if rc != SS_OK:
            if raise_on_error:
                raise SSError(rc, f"ss_graph_capture (op {res.failed_op})")
            return Graph(None, self, res)
        return Graph(g, self, res)

    def sync(self) -> _Result:
        res = _Result()
        _check(lib.ss_sync(self.h, ctypes.byref(res)), "ss_sync")
        return res

    def set_option(self, key: str, value: int):
        _check(lib.ss_set_option(self.h, key.encode(), int(value)), "ss_set_option")

    def trace(self) -> dict:
        """Per kernel category: launches, seconds (HIP events), algorithmic bytes, entries."""
        out = {}
        for i, name in enumerate(TRACE_CATS):
            n, b, e = ctypes.c_uint64(0), ctypes.c_uint64(0), ctypes.c_uint64(0)
            sec = ctypes.c_double(0.0)
            _check(lib.ss_trace_read(self.h, i, ctypes.byref(n), ctypes.byref(sec), ctypes.byref(b),
                                     ctypes.byref(e)), "ss_trace_read")
            out[name] = {"launches": int(n.value), "seconds": float(sec.value), "bytes": int(b.value),
                         "entries": int(e.value)}
        return out

    def stats(self) -> dict:
        a = (ctypes.c_uint64 * 9)()
        _check(lib.ss_stats(self.h, a), "ss_stats")
        names = ("kernels", "sort_passes", "sorts", "group_launches", "expand_launches", "perm_runs",
                 "host_syncs", "entries_updated", "speculation_wasted")
        return {k: int(v) for k, v in zip(names, a)}


class Graph:
    """A captured op list of one State (``State.capture``); ``launch`` replays it."""

    def __init__(self, handle, state: "State", result: _Result):
        self.h = handle
        self.state = state          # keeps the state (and its arena) alive
        self.result = result        # status of the applying capture call

    def launch(self, raise_on_error: bool = True) -> _Result:
        res = _Result()
        if not self.h:
            raise SSError(SS_E_ARG, "ss_graph_launch (no graph)")
        rc = lib.ss_graph_launch(self.h, ctypes.byref(res))
        res.status = rc
        if rc != SS_OK and raise_on_error:
            raise SSError(rc, f"ss_graph_launch (op {res.failed_op})")
        return res

    def close(self):
        if getattr(self, "h", None):
            lib.ss_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def state_for_circuit(c: "wl.Circuit", cap_entries: Optional[int] = None, ninst: int = 1, **kw) -> State:
    """Create a state for a circuit (registers, eps, tables, initial entries)."""
    if cap_entries is None:
        cap_entries = max(1024, 2 * (1 << (c.cap_bits or 14)))
    tb = sum(max(256, len(t.values) * 8) for t in c.tables) + 4096
    st = State(c.regs, ninst=ninst, eps=c.eps, cap_entries=cap_entries, table_bytes=tb, **kw)
    for t in c.tables:
        st.load_qram(t)
    for m in c.matrices:
        st.load_matrix(m)
    if c.init_values is not None:
        st.set_entries(0, c.init_values, c.init_amps)
    return st
