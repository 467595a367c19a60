"""A front end for a subset of OpenQASM 2.0 (the paper's benchmark circuits
are read as QASM, Sec. "Results").

Reads ``qreg`` declarations and gate applications and returns a register-level
circuit (``workloads.Circuit``) for the simulator: each ``qreg`` becomes one
register (split into registers of at most 64 qubits when longer), and each
gate becomes one op of the library's kinds.  Supported:

    x y z h s sdg t tdg id sx sxdg   rx ry rz p u1 u2 u3 u
    cx cy cz ch ccx swap cp cu1 crz cry crx cu3   barrier  measure  creg

Gates on a whole register (``h q;``) apply to each of its qubits.  Angle
expressions use numbers, ``pi``, + - * / and parentheses.  ``measure`` is
recorded (``Program.measures``), not applied.  Custom ``gate`` definitions,
``if`` and ``reset`` are outside the subset (ValueError).

Gate matrices follow the OpenQASM 2.0 definitions, row = output bit:
rz(t) = diag(e^{-it/2}, e^{it/2}); rx(t) = [[c, -is], [-is, c]] (c, s of
t/2); u3(t, f, l) = [[c, -e^{il} s], [e^{if} s, e^{i(f+l)} c]]; u2(f, l) =
u3(pi/2, f, l); p(l) = u1(l) = diag(1, e^{il}); sx = (1/2)[[1+i, 1-i],
[1-i, 1+i]].  Diagonal ones map to phase ops (no branching); rotations by
2x2 matrices use the library's ROT kind.  Parsing is host-side input
preparation: every gate runs in the library's kernels.
"""
from __future__ import annotations

import dataclasses
import math
import re
from typing import Dict, List, Tuple

import numpy as np

import workloads as wl


@dataclasses.dataclass
class Program:
    circuit: "wl.Circuit"
    qregs: Dict[str, Tuple[int, int]]          # name -> (first register index, qubits)
    measures: List[Tuple[int, int, str, int]]  # (register, qubit, creg, bit)


_TOKEN = re.compile(r"\s*(?:(\d+\.\d*(?:[eE][-+]?\d+)?|\d*\.\d+(?:[eE][-+]?\d+)?|\d+(?:[eE][-+]?\d+)?)|(pi)|(.))")


def _eval_expr(text: str) -> float:
    """Angle expression: numbers, pi, unary -, + - * /, parentheses."""
    toks = []
    for num, pi, ch in _TOKEN.findall(text):
        if num:
            toks.append(("n", float(num)))
        elif pi:
            toks.append(("n", math.pi))
        elif ch.strip():
            toks.append(("o", ch))
    pos = 0

    def peek():
        return toks[pos] if pos < len(toks) else ("e", None)

    def atom():
        nonlocal pos
        t = peek()
        if t == ("o", "-"):
            pos += 1
            return -atom()
        if t == ("o", "+"):
            pos += 1
            return atom()
        if t == ("o", "("):
            pos += 1
            v = expr()
            if peek() != ("o", ")"):
                raise ValueError(f"bad expression {text!r}")
            pos += 1
            return v
        if t[0] == "n":
            pos += 1
            return t[1]
        raise ValueError(f"bad expression {text!r}")

    def term():
        nonlocal pos
        v = atom()
        while peek() in (("o", "*"), ("o", "/")):
            op = peek()[1]
            pos += 1
            r = atom()
            v = v * r if op == "*" else v / r
        return v

    def expr():
        nonlocal pos
        v = term()
        while peek() in (("o", "+"), ("o", "-")):
            op = peek()[1]
            pos += 1
            r = term()
            v = v + r if op == "+" else v - r
        return v

    v = expr()
    if pos != len(toks):
        raise ValueError(f"bad expression {text!r}")
    return v


def _u3(t, f, l):
    c, s = math.cos(t / 2), math.sin(t / 2)
    return np.array([[c, -np.exp(1j * l) * s], [np.exp(1j * f) * s, np.exp(1j * (f + l)) * c]],
                    dtype=np.complex128)


def _matrix(name, args):
    if name == "rz":
        t = args[0]
        return np.diag([np.exp(-0.5j * t), np.exp(0.5j * t)]).astype(np.complex128)
    if name == "rx":
        c, s = math.cos(args[0] / 2), math.sin(args[0] / 2)
        return np.array([[c, -1j * s], [-1j * s, c]], dtype=np.complex128)
    if name in ("u3", "u", "cu3"):
        return _u3(*args)
    if name == "u2":
        return _u3(math.pi / 2, args[0], args[1])
    if name == "sx":
        return 0.5 * np.array([[1 + 1j, 1 - 1j], [1 - 1j, 1 + 1j]], dtype=np.complex128)
    if name == "sxdg":
        return 0.5 * np.array([[1 - 1j, 1 + 1j], [1 + 1j, 1 - 1j]], dtype=np.complex128)
    raise KeyError(name)


_ONE = {"x": "X", "y": "Y", "z": "Z", "h": "H", "s": "S", "sdg": "SDG", "t": "T", "tdg": "TDG"}
_CTRL = {"cx": "X", "cy": "Y", "cz": "Z", "ch": "H", "ccx": "X"}


def parse(text: str, eps: float = 1e-14, name: str = "qasm") -> Program:
    # strip comments, split statements
    text = re.sub(r"//[^\n]*", "", text)
    stmts = [s.strip() for s in text.split(";") if s.strip()]
    regs: List[Tuple[str, int]] = []
    qregs: Dict[str, Tuple[int, int]] = {}
    ops = []
    mats: List[np.ndarray] = []
    measures = []

    def qubits(arg: str) -> List[Tuple[int, int]]:
        """(register, qubit) of 'q[i]', or of every qubit of 'q'."""
        m = re.fullmatch(r"([A-Za-z_]\w*)\s*(?:\[\s*(\d+)\s*\])?", arg.strip())
        if not m or m.group(1) not in qregs:
            raise ValueError(f"unknown qubit {arg!r}")
        first, n = qregs[m.group(1)]
        idx = [int(m.group(2))] if m.group(2) is not None else list(range(n))
        out = []
        for i in idx:
            if i >= n:
                raise ValueError(f"qubit {arg!r} out of range")
            out.append((first + i // 64, i % 64))
        return out

    def matrix_id(m: np.ndarray) -> int:
        for j, x in enumerate(mats):
            if np.array_equal(x, m):
                return j
        mats.append(m)
        return len(mats) - 1

    for st in stmts:
        if st.startswith("OPENQASM") or st.startswith("include"):
            continue
        m = re.fullmatch(r"qreg\s+([A-Za-z_]\w*)\s*\[\s*(\d+)\s*\]", st)
        if m:
            n = int(m.group(2))
            if n < 1:
                raise ValueError("empty qreg")
            qregs[m.group(1)] = (len(regs), n)
            for j in range(0, n, 64):
                regs.append((m.group(1) if n <= 64 else f"{m.group(1)}.{j // 64}", min(64, n - j)))
            continue
        if st.startswith("creg") or st.startswith("barrier"):
            continue
        m = re.fullmatch(r"measure\s+(.+?)\s*->\s*([A-Za-z_]\w*)\s*(?:\[\s*(\d+)\s*\])?", st)
        if m:
            qs = qubits(m.group(1))
            for j, (r, q) in enumerate(qs):
                measures.append((r, q, m.group(2), int(m.group(3)) if m.group(3) is not None else j))
            continue
        m = re.fullmatch(r"([A-Za-z_]\w*)\s*(?:\((.*)\))?\s+(.+)", st, flags=re.S)
        if not m:
            raise ValueError(f"cannot parse {st!r}")
        g, argtext, qtext = m.group(1), m.group(2), m.group(3)
        if g in ("gate", "opaque", "if", "reset"):
            raise ValueError(f"'{g}' is outside the supported subset")
        args = [_eval_expr(a) for a in argtext.split(",")] if argtext else []
        operands = [qubits(a) for a in qtext.split(",")]
        if len(operands) > 1:
            # broadcast: registers of equal length pair up qubit by qubit
            L = max(len(o) for o in operands)
            operands = [o * L if len(o) == 1 else o for o in operands]
            if any(len(o) != L for o in operands):
                raise ValueError(f"operand lengths differ in {st!r}")
        apps = list(zip(*operands))
        for qs in apps:
            ops.extend(_gate_ops(g, args, qs, matrix_id))
    c = wl.Circuit(regs=regs, ops=wl.ops_array(ops), eps=eps, matrices=mats, name=name)
    return Program(circuit=c, qregs=qregs, measures=measures)


def _gate_ops(g, args, qs, matrix_id):
    def one(kind, q, ctls=(), **kw):
        return wl.make_op(kind, q[0], qmask=1 << q[1], ctls=[(r, b, 1) for r, b in ctls], **kw)

    if g == "id":
        return []
    if g in _ONE:
        return [one(_ONE[g], qs[0])]
    if g == "ry":
        return [one("RY", qs[0], theta=args[0])]
    if g in ("p", "u1"):
        return [one("PHASE", qs[0], theta=args[0])]
    if g in ("rz", "rx", "u3", "u", "u2", "sx", "sxdg"):
        return [one("ROT", qs[0], table=matrix_id(_matrix(g, args)))]
    if g in _CTRL:
        return [one(_CTRL[g], qs[-1], ctls=qs[:-1])]
    if g in ("cp", "cu1"):
        return [one("PHASE", qs[1], ctls=[qs[0]], theta=args[0])]
    if g == "cry":
        return [one("RY", qs[1], ctls=[qs[0]], theta=args[0])]
    if g in ("crz", "crx", "cu3"):
        base = {"crz": "rz", "crx": "rx", "cu3": "cu3"}[g]
        return [one("ROT", qs[1], ctls=[qs[0]], table=matrix_id(_matrix(base, args)))]
    if g == "swap":
        a, b = qs
        return [one("X", b, ctls=[a]), one("X", a, ctls=[b]), one("X", b, ctls=[a])]
    raise ValueError(f"gate '{g}' is outside the supported subset")


def to_qasm(c: "wl.Circuit") -> str:
    """OpenQASM 2.0 text of a circuit built from the gates this front end
    reads (registers of one qubit-index space each; used by tests)."""
    lines = ["OPENQASM 2.0;", 'include "qelib1.inc";']
    for name, w in c.regs:
        lines.append(f"qreg {name}[{w}];")
    names = [n for n, _ in c.regs]
    inv = {v: k for k, v in _ONE.items()}
    for op in c.ops:
        kind = wl.KINDS[int(op["kind"])]
        r = int(op["reg"])
        qbits = [q for q in range(64) if (int(op["qmask"]) >> q) & 1]
        ctls = [(int(op["ctl_reg"][j]), int(op["ctl_qubit"][j]), int(op["ctl_val"][j])) for j in range(int(op["nctl"]))]
        if any(v != 1 for _, _, v in ctls):
            raise ValueError("QASM controls are on |1>")
        cq = [f"{names[x]}[{b}]" for x, b, _ in ctls]
        for q in qbits:
            t = f"{names[r]}[{q}]"
            if kind in inv and not ctls:
                lines.append(f"{inv[kind]} {t};")
            elif kind == "X" and len(ctls) in (1, 2):
                lines.append(("cx " if len(ctls) == 1 else "ccx ") + ", ".join(cq + [t]) + ";")
            elif kind in ("Y", "Z", "H") and len(ctls) == 1:
                lines.append(f"c{kind.lower()} {cq[0]}, {t};")
            elif kind == "RY":
                lines.append((f"cry({float(op['theta'])!r}) {cq[0]}, " if ctls else f"ry({float(op['theta'])!r}) ") + t + ";")
            elif kind == "PHASE":
                lines.append((f"cp({float(op['theta'])!r}) {cq[0]}, " if ctls else f"p({float(op['theta'])!r}) ") + t + ";")
            else:
                raise ValueError(f"no QASM form for {kind} with {len(ctls)} controls")
    return "\n".join(lines) + "\n"
