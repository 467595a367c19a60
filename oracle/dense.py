"""Dense brute-force state-vector checker (test infrastructure only).

A second, independent CPU reference used to pin the sparse oracle on circuits
of at most ~22 qubits.  The state is a complex128 numpy vector indexed by the
flat basis index  sum_r value_r << (width_0 + ... + width_{r-1})  (register 0
in the lowest bits), i.e. the Kronecker-product basis of the section "Qubits
and quantum operations" with qubit q of a register as bit q of its value.

* permutation ops (X, ADD, SUB, MULC, XOR, XORC, QRAM load/unload) move every
  amplitude to f(index) through an index array; the map is checked to be a
  bijection (QRAM equation; non-interference ops);
* REFLECT0 multiplies by +i / -i (the QLSS reflection R);
* Y, Z, S, S^-1, T, T^-1 and diag(1, e^{i theta}) (Sec. "Qubits and quantum
  operations"; phase gates among the non-interference ops) and ROT (a 2x2
  complex matrix, the supplementary Rot_Int) update each (bit=0, bit=1) pair
  with their matrix where the controls hold, one qubit at a time; only a ROT
  whose matrix is neither diagonal nor off-diagonal is followed by the
  clear-zero step;
* ADDC, MUL, DIV (register arithmetic oracles) are permutations like ADD;
* H and Ry update each (bit=0, bit=1) pair with the 2x2 matrix where the
  controls hold (controlled-U definition), one target qubit at a time in
  ascending order, and after the whole op every amplitude with
  |a|^2 < eps^2 is set to zero (clear-zero step of interference ops).
"""
from __future__ import annotations

import numpy as np

import workloads as wl

C_H = 0.70710678118654752440


class DenseState:
    def __init__(self, regs, eps=1e-14, tables=(), init_values=None, init_amps=None, matrices=()):
        self.widths = [int(w) for _, w in regs]
        self.offs = np.cumsum([0] + self.widths[:-1]).tolist()
        self.nq = sum(self.widths)
        if self.nq > 24:
            raise ValueError("dense checker is limited to 24 qubits")
        self.eps = float(eps)
        self.tables = list(tables)
        self.matrices = [np.asarray(m, dtype=np.complex128).reshape(2, 2) for m in matrices]
        self.v = np.zeros(1 << self.nq, dtype=np.complex128)
        self.idx = np.arange(1 << self.nq, dtype=np.uint64)
        if init_values is None:
            self.v[0] = 1.0
        else:
            flat = self.flat_of(np.asarray(init_values, dtype=np.uint64))
            self.v[flat] = np.asarray(init_amps, dtype=np.complex128)

    @classmethod
    def from_circuit(cls, c: "wl.Circuit") -> "DenseState":
        return cls(c.regs, c.eps, c.tables, c.init_values, c.init_amps, c.matrices)

    def flat_of(self, values: np.ndarray) -> np.ndarray:
        out = np.zeros(values.shape[0], dtype=np.uint64)
        for r, (o, w) in enumerate(zip(self.offs, self.widths)):
            out |= (values[:, r] & np.uint64((1 << w) - 1)) << np.uint64(o)
        return out.astype(np.int64)

    def field(self, idx, r):
        return (idx >> np.uint64(self.offs[r])) & np.uint64((1 << self.widths[r]) - 1)

    def with_field(self, idx, r, val):
        m = np.uint64(((1 << self.widths[r]) - 1) << self.offs[r])
        return (idx & ~m) | ((val << np.uint64(self.offs[r])) & m)

    def ctrl(self, op, idx):
        ok = np.ones(idx.shape, dtype=bool)
        for j in range(int(op["nctl"])):
            r = int(op["ctl_reg"][j])
            q = int(op["ctl_qubit"][j])
            bit = (idx >> np.uint64(self.offs[r] + q)) & np.uint64(1)
            ok &= bit == np.uint64(op["ctl_val"][j])
        return ok

    def apply(self, ops):
        for op in ops:
            self.apply_op(op)

    def apply_op(self, op):
        kind = wl.KINDS[int(op["kind"])]
        r = int(op["reg"])
        w = self.widths[r]
        wm = np.uint64((1 << w) - 1)
        idx = self.idx
        on = self.ctrl(op, idx)
        if kind in ("H", "RY"):
            if kind == "H":
                m = np.array([[C_H, C_H], [C_H, -C_H]])
            else:
                h = float(op["theta"]) / 2.0
                m = np.array([[np.cos(h), -np.sin(h)], [np.sin(h), np.cos(h)]])
            for q in range(w):
                if not (int(op["qmask"]) >> q) & 1:
                    continue
                bit = np.uint64(1 << (self.offs[r] + q))
                i0 = idx[((idx & bit) == 0) & on].astype(np.int64)
                i1 = (i0.astype(np.uint64) | bit).astype(np.int64)
                a0 = self.v[i0].copy()
                a1 = self.v[i1].copy()
                # real matrix elements times complex amplitudes, component-wise
                self.v[i0] = _rmul(m[0, 0], a0) + _rmul(m[0, 1], a1)
                self.v[i1] = _rmul(m[1, 0], a0) + _rmul(m[1, 1], a1)
            a2 = self.v.real * self.v.real + self.v.imag * self.v.imag
            self.v[a2 < self.eps * self.eps] = 0.0
            return
        mats = {"Y": [[0, -1j], [1j, 0]], "Z": [[1, 0], [0, -1]], "S": [[1, 0], [0, 1j]],
                "SDG": [[1, 0], [0, -1j]], "T": [[1, 0], [0, complex(C_H, C_H)]],
                "TDG": [[1, 0], [0, complex(C_H, -C_H)]]}
        if kind in mats or kind in ("PHASE", "ROT"):
            if kind == "PHASE":
                m = np.array([[1, 0], [0, complex(np.cos(float(op["theta"])), np.sin(float(op["theta"])))]])
            elif kind == "ROT":
                m = self.matrices[int(op["table"])]
            else:
                m = np.array(mats[kind], dtype=np.complex128)
            for q in range(w):
                if not (int(op["qmask"]) >> q) & 1:
                    continue
                bit = np.uint64(1 << (self.offs[r] + q))
                i0 = idx[((idx & bit) == 0) & on].astype(np.int64)
                i1 = (i0.astype(np.uint64) | bit).astype(np.int64)
                a0 = self.v[i0].copy()
                a1 = self.v[i1].copy()
                self.v[i0] = m[0, 0] * a0 + m[0, 1] * a1
                self.v[i1] = m[1, 0] * a0 + m[1, 1] * a1
            one_to_one = (m[0, 1] == 0 and m[1, 0] == 0) or (m[0, 0] == 0 and m[1, 1] == 0)
            if not one_to_one:
                a2 = self.v.real * self.v.real + self.v.imag * self.v.imag
                self.v[a2 < self.eps * self.eps] = 0.0
            return
        if kind == "REFLECT0":
            z = self.field(idx, r) == 0
            ph = np.where(z, 1j, -1j)
            self.v = np.where(on, self.v * ph, self.v)
            return
        val = self.field(idx, r)
        if kind == "X":
            new = val ^ (np.uint64(op["qmask"]) & wm)
        elif kind in ("ADD", "SUB", "XOR"):
            src = self.field(idx, int(op["reg2"])) & wm
            if kind == "ADD":
                new = (val + src) & wm
            elif kind == "SUB":
                new = (val - src) & wm
            else:
                new = val ^ src
        elif kind == "MULC":
            new = (val * np.uint64(op["imm"])) & wm
        elif kind == "XORC":
            new = val ^ (np.uint64(op["imm"]) & wm)
        elif kind == "ADDC":
            new = (val + (np.uint64(op["imm"]) & wm)) & wm
        elif kind == "MUL":
            x = self.field(idx, int(op["reg2"]))
            y = self.field(idx, int(op["reg3"]))
            with np.errstate(over="ignore"):
                new = (val ^ (x * y)) & wm
        elif kind == "DIV":
            x = self.field(idx, int(op["reg2"]))
            y = self.field(idx, int(op["reg3"]))
            r4 = int(op["reg4"])
            wm4 = np.uint64((1 << self.widths[r4]) - 1)
            ysafe = np.where(y == 0, np.uint64(1), y)
            quo = np.where(y == 0, ~np.uint64(0), x // ysafe)
            rem = np.where(y == 0, x, x % ysafe)
            new = (val ^ quo) & wm
            nr4 = (self.field(idx, r4) ^ rem) & wm4
            idx = self.with_field(idx, r4, nr4)
            dst = np.where(on, self.with_field(idx, r, new), self.idx).astype(np.int64)
            if len(np.unique(dst)) != len(dst):
                raise AssertionError("permutation op is not a bijection")
            out = np.zeros_like(self.v)
            out[dst] = self.v
            self.v = out
            return
        elif kind in ("QRAM_LOAD", "QRAM_UNLOAD"):
            t = self.tables[int(op["table"])]
            addr = self.field(idx, int(op["reg2"])).astype(np.int64)
            new = (val ^ np.asarray(t.values, dtype=np.uint64)[addr]) & wm
        else:
            raise ValueError(kind)
        dst = np.where(on, self.with_field(idx, r, new), idx).astype(np.int64)
        if len(np.unique(dst)) != len(dst):
            raise AssertionError("permutation op is not a bijection")
        out = np.zeros_like(self.v)
        out[dst] = self.v
        self.v = out

    def entries(self):
        """(values[n, nregs] uint64, amps[n]) of the nonzero entries, ascending flat index."""
        nz = np.nonzero(self.v)[0]
        vals = np.zeros((len(nz), len(self.widths)), dtype=np.uint64)
        u = nz.astype(np.uint64)
        for r in range(len(self.widths)):
            vals[:, r] = self.field(u, r)
        return vals, self.v[nz]


def _rmul(c: float, a: np.ndarray) -> np.ndarray:
    """Real matrix element times complex amplitudes, one product per component."""
    out = np.empty_like(a)
    out.real = c * a.real
    out.imag = c * a.imag
    return out
