"""Closed forms of structured workloads (test infrastructure only).

Only tests may import this module.  Like the std::map oracle it shares nothing
with the HIP path: it evaluates what the method must produce for circuits
whose structure gives the result in closed form, with vectorised numpy, at
sizes where the map oracle would take minutes.  Each function is pinned
against the map oracle on smaller instances of the same form
(tests/test_oracle_pins.py).

Key packing follows the oracle's rule: qubit q of a register is bit q of its
value, registers are placed in creation order into 64-bit words, first fit,
never straddling a word.
"""
from __future__ import annotations

import numpy as np

import workloads as wl

C = 0.70710678118654752440   # 1/sqrt(2), the H matrix element


def packing(widths):
    """(word, offset) of each register under the first-fit rule."""
    fill = [0, 0, 0, 0]
    out = []
    for w in widths:
        word = 0
        while fill[word] + w > 64:
            word += 1
        out.append((word, fill[word]))
        fill[word] += w
    return out


def _ry(theta):
    c, s = np.cos(theta / 2.0), np.sin(theta / 2.0)
    return np.array([[c, -s], [s, c]])


def c2_closed_form(c: "wl.Circuit", eps_margin: float = 1e-10):
    """The arithmetic-heavy circuit (registers a, b, c of 32 qubits and a
    1-qubit flag; H on some qubits of a, then register arithmetic, X with
    controls and Ry, or a rotation by a 2x2 complex matrix, on the flag only).

    Each initial value of a follows one classical trajectory through the
    permutation ops (Sec. "Non-interference operations": every branch is
    rewritten on its own), and the flag is never read by them, so the final
    state is sum over the 2^h start values s of |traj(s)> (x) c^h Ry...Ry|0>.
    Returns (keys[n, 2] uint64 ascending, amps[n] complex128).

    The prune after each Ry removes a flag component below eps; the closed form
    assumes none comes within ``eps_margin`` of it (checked)."""
    widths = [w for _, w in c.regs]
    assert widths == [32, 32, 32, 1]
    ops = c.ops
    assert wl.KINDS[int(ops[0]["kind"])] == "H" and int(ops[0]["reg"]) == 0 and int(ops[0]["nctl"]) == 0
    hmask = int(ops[0]["qmask"])
    qs = [q for q in range(32) if (hmask >> q) & 1]
    h = len(qs)
    idx = np.arange(2 ** h, dtype=np.uint64)
    a = np.zeros(2 ** h, dtype=np.uint64)
    for j, q in enumerate(qs):
        a |= ((idx >> np.uint64(j)) & np.uint64(1)) << np.uint64(q)
    regs = [a, np.zeros_like(a), np.zeros_like(a)]
    M = np.uint64(0xFFFFFFFF)
    amp0 = 1.0
    for _ in range(h):
        amp0 = C * amp0
    vec = np.array([amp0, 0.0], dtype=np.complex128)
    for op in ops[1:]:
        kind = wl.KINDS[int(op["kind"])]
        d = int(op["reg"])
        if kind in ("RY", "ROT"):
            assert d == 3 and int(op["nctl"]) == 0
            m = _ry(float(op["theta"])) if kind == "RY" else np.asarray(c.matrices[int(op["table"])])
            vec = m @ vec
            small = np.abs(vec)[np.abs(vec) > 0]
            assert not np.any(np.abs(small - c.eps) < eps_margin) and not np.any(
                (small < c.eps) & (small > 0)), "a flag amplitude near the prune threshold"
            continue
        assert d < 3
        s = int(op["reg2"])
        if kind == "ADD":
            regs[d] = (regs[d] + regs[s]) & M
        elif kind == "SUB":
            regs[d] = (regs[d] - regs[s]) & M
        elif kind == "MULC":
            with np.errstate(over="ignore"):
                regs[d] = (regs[d] * np.uint64(int(op["imm"]) & 0xFFFFFFFF)) & M
        elif kind == "XOR":
            regs[d] = regs[d] ^ regs[s]
        elif kind == "XORC":
            regs[d] = regs[d] ^ (np.uint64(int(op["imm"])) & M)
        elif kind == "X":
            on = np.ones(len(a), dtype=bool)
            for j in range(int(op["nctl"])):
                r, q, v = int(op["ctl_reg"][j]), int(op["ctl_qubit"][j]), int(op["ctl_val"][j])
                on &= ((regs[r] >> np.uint64(q)) & np.uint64(1)) == np.uint64(v)
            regs[d] = np.where(on, regs[d] ^ (np.uint64(int(op["qmask"])) & M), regs[d])
        else:
            raise ValueError(f"kind {kind} is not part of the arithmetic-heavy form")
    lay = packing(widths)
    assert lay == [(0, 0), (0, 32), (1, 0), (1, 32)]
    w0 = regs[0] | (regs[1] << np.uint64(32))
    keys, amps = [], []
    for f in (0, 1):
        if abs(vec[f]) ** 2 < c.eps * c.eps or vec[f] == 0.0:
            continue
        w1 = regs[2] | (np.uint64(f) << np.uint64(32))
        keys.append(np.stack([w0, w1], axis=1))
        amps.append(np.full(len(a), vec[f], dtype=np.complex128))
    keys = np.concatenate(keys)
    amps = np.concatenate(amps)
    order = np.lexsort((keys[:, 0], keys[:, 1]))
    return keys[order], amps[order]
