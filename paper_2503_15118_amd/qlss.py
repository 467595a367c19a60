"""Building blocks of the QRAM-based linear-system solver as op lists.

The block encoding of a matrix A is reduced to controlled state preparation
(supplementary section on the linear-system solver with QRAM):

    U_A = U_SWAP U_R^dagger U_L,
    U_L |k>|0>|0> = |k>|0>|phi_k>,  phi_k = sum_j A_jk / ||A_.k|| |j>,
    U_R |0>|0>|j> = |psi>|0>|j>,    psi   = sum_k ||A_.k|| / ||A||_F |k>,
    U_SWAP |i>|0>|j> = |j>|0>|i>,

so that <i|<0|<0| U_A |j>|0>|0> = A_ij / ||A||_F (Frobenius norm).  The state
preparations rotate one qubit per level of a binary tree (most significant
qubit first) by an angle read from QRAM, addressed by the column k and the
qubits already prepared; the walk step applies the reflection
R = i(2|0><0|_anc - I) (x) I of the same section after U_A.

Layout: registers t (n qubits: column / row index), d (w qubits: the QRAM
word, a w-bit two's-complement angle theta = pi q / 2^(w-2)), b (n qubits:
the prepared state) and a (2n qubits: the QRAM address: k in its low n bits,
the prepared prefix above).  d and a return to 0 after every block.

A rotation by an angle held in d is applied as w rotations of b's qubit, one
per bit of d (controlled by that bit), with angles pi 2^(j - w + 2) and -2 pi
for the sign bit; their product is Ry(pi q / 2^(w-2)) exactly in exact
arithmetic.  This module only builds tables and op lists (host-side input
preparation); every op runs in the library's kernels.
"""
from __future__ import annotations

import dataclasses
from typing import List

import numpy as np

import workloads as wl

T, D, B, A = 0, 1, 2, 3          # register indices


@dataclasses.dataclass
class BlockEncoding:
    n: int                       # qubits of t and b (A is 2^n x 2^n)
    w: int                       # bits of an angle word
    regs: list
    tables: List["wl.Table"]     # U_L levels 0..n-1, then U_R levels 0..n-1
    fro: float                   # ||A||_F
    ul: np.ndarray               # op lists
    ur: np.ndarray
    ua: np.ndarray


def quantize(theta, w: int) -> np.ndarray:
    """theta (radians, in [-2 pi, 2 pi]) as a w-bit two's-complement word q
    with theta = pi q / 2^(w-2), rounded to nearest; 2 pi wraps to -2 pi,
    the same rotation (Ry(2 pi) = Ry(-2 pi) = -I)."""
    q = np.rint(np.asarray(theta, dtype=np.float64) / np.pi * 2.0 ** (w - 2)).astype(np.int64)
    return (q & ((1 << w) - 1)).astype(np.uint64)


def dequantize(q, w: int) -> np.ndarray:
    q = np.asarray(q, dtype=np.int64)
    q = np.where(q >= 2 ** (w - 1), q - 2 ** w, q)
    return np.pi * q.astype(np.float64) / 2.0 ** (w - 2)


def tree_angles(v: np.ndarray) -> List[np.ndarray]:
    """Binary-tree angles preparing the real vector v (length 2^n, nonzero)
    up to its norm: level l (0 = most significant qubit) has 2^l angles, one
    per prefix p of the l qubits above; rotating qubit n-1-l by Ry(theta)
    splits the prefix's weight between its two halves.  The last level takes
    signed leaves, so signs of v are reproduced."""
    v = np.asarray(v, dtype=np.float64)
    n = int(np.log2(len(v)))
    out = []
    for l in range(n):
        half = 2 ** (n - 1 - l)
        blocks = v.reshape(2 ** l, 2, half)        # prefix, this qubit, rest
        if l == n - 1:
            th = 2.0 * np.arctan2(blocks[:, 1, 0], blocks[:, 0, 0])
        else:
            th = 2.0 * np.arctan2(np.linalg.norm(blocks[:, 1, :], axis=1), np.linalg.norm(blocks[:, 0, :], axis=1))
        out.append(th)
    return out


def _addr(n: int, l: int, k, prefix):
    """Address of level l: k in bits 0..n-1 and prefix bit i (the qubit
    n-1-i of the prepared register, i < l) in bit n+i."""
    a = np.uint64(k)
    for i in range(l):
        a |= np.uint64((int(prefix) >> (l - 1 - i)) & 1) << np.uint64(n + i)
    return a


def _tables(Amat: np.ndarray, w: int):
    n = int(np.log2(Amat.shape[0]))
    N = 2 ** n
    col = np.linalg.norm(Amat, axis=0)
    fro = float(np.linalg.norm(Amat))
    tl = [np.zeros(2 ** (2 * n), dtype=np.uint64) for _ in range(n)]
    tr = [np.zeros(2 ** (2 * n), dtype=np.uint64) for _ in range(n)]
    for k in range(N):
        if col[k] == 0.0:
            continue
        for l, th in enumerate(tree_angles(Amat[:, k])):
            q = quantize(th, w)
            for p in range(2 ** l):
                tl[l][int(_addr(n, l, k, p))] = q[p]
    for l, th in enumerate(tree_angles(col / fro)):
        q = quantize(th, w)
        for p in range(2 ** l):
            tr[l][int(_addr(n, l, 0, p))] = q[p]
    tabs = [wl.Table(values=t, addr_bits=2 * n, word_bits=w) for t in tl + tr]
    return n, fro, tabs


def _copy_prefix(n: int, l: int, src: int):
    """X on address qubits n+i controlled by qubit n-1-i of `src` (i < l)."""
    return [wl.make_op("X", A, qmask=1 << (n + i), ctls=[(src, n - 1 - i, 1)]) for i in range(l)]


def _rot_by_word(w: int, reg: int, qubit: int, sign: float = 1.0):
    """Ry(pi q / 2^(w-2)) on one qubit, q the word in d: one rotation per bit."""
    ops = []
    for j in range(w):
        ang = -2.0 * np.pi if j == w - 1 else np.pi * 2.0 ** (j - (w - 2))
        ops.append(wl.make_op("RY", reg, qmask=1 << qubit, theta=sign * ang, ctls=[(D, j, 1)]))
    return ops


def _prep(n: int, w: int, target: int, table0: int, with_k: bool):
    ops = []
    if with_k:
        ops.append(wl.make_op("XOR", A, reg2=T))
    for l in range(n):
        ops += _copy_prefix(n, l, target)
        ops.append(wl.make_op("QRAM_LOAD", D, reg2=A, table=table0 + l))
        ops += _rot_by_word(w, target, n - 1 - l)
        ops.append(wl.make_op("QRAM_UNLOAD", D, reg2=A, table=table0 + l))
        ops += _copy_prefix(n, l, target)
    if with_k:
        ops.append(wl.make_op("XOR", A, reg2=T))
    return ops


def _inverse(ops):
    """The inverse of a list of X / XOR / QRAM / RY ops: reversed, each Ry
    angle negated (the others are their own inverses)."""
    out = []
    for op in reversed(ops):
        o = op.copy()
        if wl.KINDS[int(o["kind"])] == "RY":
            o["theta"] = -float(o["theta"])
        elif wl.KINDS[int(o["kind"])] not in ("X", "XOR", "QRAM_LOAD", "QRAM_UNLOAD"):
            raise ValueError("no inverse for this kind")
        out.append(o)
    return out


def block_encoding(Amat: np.ndarray, w: int = 32) -> BlockEncoding:
    """Tables and op lists of U_L, U_R and U_A for a real 2^n x 2^n matrix."""
    n, fro, tabs = _tables(np.asarray(Amat, dtype=np.float64), w)
    regs = [("t", n), ("d", w), ("b", n), ("a", 2 * n)]
    ul = _prep(n, w, B, 0, True)
    ur = _prep(n, w, T, n, False)
    swap = [wl.make_op("XOR", T, reg2=B), wl.make_op("XOR", B, reg2=T), wl.make_op("XOR", T, reg2=B)]
    ua = ul + _inverse(ur) + swap
    return BlockEncoding(n=n, w=w, regs=regs, tables=tabs, fro=fro,
                         ul=wl.ops_array(ul), ur=wl.ops_array(ur), ua=wl.ops_array(ua))


def walk_step(be: BlockEncoding) -> np.ndarray:
    """One step of the qubitised walk W = R U_A, R the reflection about
    |0> of the ancilla register b (d and a are 0 between blocks)."""
    return np.concatenate([be.ua, wl.ops_array([wl.make_op("REFLECT0", B)])])


def circuit(be: BlockEncoding, ops: np.ndarray, j=None, amps=None, eps: float = 1e-14,
            name: str = "qlss") -> "wl.Circuit":
    """A circuit on the block encoding's registers starting from |j>_t (or
    the superposition sum_j amps_j |j>_t), the other registers 0."""
    if j is None and amps is None:
        j = 0
    if amps is None:
        vals = np.array([[j, 0, 0, 0]], dtype=np.uint64)
        a = np.array([1.0 + 0j])
    else:
        nz = np.flatnonzero(amps)
        vals = np.zeros((len(nz), 4), dtype=np.uint64)
        vals[:, 0] = nz
        a = np.asarray(amps, dtype=np.complex128)[nz]
    return wl.Circuit(regs=be.regs, ops=ops, eps=eps, tables=be.tables, init_values=vals, init_amps=a,
                      cap_bits=2 * be.n + 1, name=name)
