"""Seeded synthetic workloads for the sparse register-level simulator.

This module only *describes* inputs: register widths, op lists, QRAM tables and
initial entries, all drawn from ``numpy.random.Generator(PCG64(seed))``.  It
holds none of the simulation arithmetic (no key packing, no gate matrices, no
amplitude updates), so both the HIP path and the CPU oracle can consume its
output without sharing any of the method's code.

Register-level state (Sec. "Sparse state representation and data structure"):
a state is a sum of branches a_i |v^0_i>|v^1_i>...; an op list is a sequence of
register-level operations (non-interference ops of the section "Non-interference
operations", interference ops of "Interference operations", QRAM of the QRAM
section's defining equation, and the reflection R of the QLSS section).

Op records use ``OP_DTYPE``.  Field meaning per kind:

* ``X``      flip every qubit of ``qmask`` in register ``reg``.
* ``H``      Hadamard on every qubit of ``qmask`` in ``reg`` (ascending qubit order).
* ``RY``     Ry(theta) on the single qubit of ``qmask`` in ``reg``.
* ``ADD``/``SUB``  reg <- reg +/- reg2  (mod 2^width(reg)).
* ``MULC``   reg <- reg * imm (mod 2^width(reg)), imm odd.
* ``XOR``    reg <- reg ^ reg2 ;  ``XORC``: reg <- reg ^ imm.
* ``QRAM_LOAD``/``QRAM_UNLOAD``  reg (data) <- reg ^ table[reg2 (address)].
* ``REFLECT0``  amplitude *= +i if register ``reg`` is 0, else -i.

Further gates of Sec. "Qubits and quantum operations" / "Non-interference
operations" and the general single-qubit rotation of the supplementary
details of quantum operations (Rot_Int):

* ``Y``, ``Z``, ``S``, ``SDG``, ``T``, ``TDG`` on every qubit of ``qmask``;
  ``PHASE`` diag(1, e^{i theta}) on every qubit of ``qmask``.
* ``ROT``    the 2x2 complex matrix ``Circuit.matrices[table]`` on the single
  qubit of ``qmask``.
* ``ADDC``   reg <- reg + imm (mod 2^width(reg)).
* ``MUL``    reg <- reg ^ (reg2 * reg3 mod 2^width(reg)).
* ``DIV``    reg <- reg ^ (reg2 div reg3), reg4 <- reg4 ^ (reg2 mod reg3).

Up to three controls ``(ctl_reg[j], ctl_qubit[j], ctl_val[j])`` gate any op.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence, Tuple

import numpy as np

BASE_KINDS = ("X", "H", "RY", "ADD", "SUB", "MULC", "XOR", "XORC",
              "QRAM_LOAD", "QRAM_UNLOAD", "REFLECT0")
EXT_KINDS = ("Y", "Z", "S", "SDG", "T", "TDG", "PHASE", "ROT", "ADDC", "MUL", "DIV")
KINDS = BASE_KINDS + EXT_KINDS
KIND = {name: i for i, name in enumerate(KINDS)}
BRANCHING = (KIND["H"], KIND["RY"])

OP_DTYPE = np.dtype([
    ("kind", "u1"), ("nctl", "u1"),
    ("reg", "u4"), ("reg2", "u4"), ("table", "u4"),
    ("qmask", "u8"), ("imm", "u8"), ("theta", "f8"),
    ("ctl_reg", "u4", (3,)), ("ctl_qubit", "u2", (3,)), ("ctl_val", "u1", (3,)),
    ("reg3", "u4"), ("reg4", "u4"),
])


@dataclasses.dataclass
class Table:
    """A QRAM memory: ``values[i]`` is d_i, ``addr_bits`` and ``word_bits`` its lengths."""
    values: np.ndarray            # uint64, len == 2**addr_bits
    addr_bits: int
    word_bits: int


@dataclasses.dataclass
class Circuit:
    """One simulation instance.

    ``init_values`` (n x nregs uint64 register values) and ``init_amps``
    (complex128) give the starting branches; ``None`` means |0...0> with
    amplitude 1.
    """
    regs: List[Tuple[str, int]]
    ops: np.ndarray
    eps: float = 1e-14
    tables: List[Table] = dataclasses.field(default_factory=list)
    init_values: Optional[np.ndarray] = None
    init_amps: Optional[np.ndarray] = None
    cap_bits: Optional[int] = None   # generator's bound: peak nnz <= 2**cap_bits
    name: str = ""
    matrices: List[np.ndarray] = dataclasses.field(default_factory=list)  # 2x2 complex (ROT)

    @property
    def nqubits(self) -> int:
        return sum(w for _, w in self.regs)

    def reg_index(self, name: str) -> int:
        return [n for n, _ in self.regs].index(name)


def make_op(kind: str, reg: int, *, qmask: int = 0, reg2: int = 0, table: int = 0,
            imm: int = 0, theta: float = 0.0,
            ctls: Sequence[Tuple[int, int, int]] = (), reg3: int = 0, reg4: int = 0) -> np.ndarray:
    rec = np.zeros((), dtype=OP_DTYPE)
    rec["kind"] = KIND[kind]
    rec["reg"] = reg
    rec["reg2"] = reg2
    rec["reg3"] = reg3
    rec["reg4"] = reg4
    rec["table"] = table
    rec["qmask"] = np.uint64(qmask)
    rec["imm"] = np.uint64(imm)
    rec["theta"] = theta
    if len(ctls) > 3:
        raise ValueError("at most 3 controls")
    rec["nctl"] = len(ctls)
    for j, (r, q, v) in enumerate(ctls):
        rec["ctl_reg"][j] = r
        rec["ctl_qubit"][j] = q
        rec["ctl_val"][j] = v
    return rec


def ops_array(recs: Sequence[np.ndarray]) -> np.ndarray:
    out = np.zeros(len(recs), dtype=OP_DTYPE)
    for i, r in enumerate(recs):
        out[i] = r
    return out


def _rng(seed) -> np.random.Generator:
    if isinstance(seed, np.random.SeedSequence):
        return np.random.Generator(np.random.PCG64(seed))
    return np.random.Generator(np.random.PCG64(int(seed)))


# ---------------------------------------------------------------------------
# C1-form: 20-qubit key (a:7, b:7, anc:6), 300 ops, peak nnz <= 2**cap_bits.
# ---------------------------------------------------------------------------
def c1_circuit(seed, nops: int = 300, cap_bits: int = 14) -> Circuit:
    """Plain smallest workload: H on up to 5 qubits of ``a``, CNOT/Toffoli on
    random qubits, ``b += a`` and Ry on an ``anc`` qubit controlled by a qubit
    of ``a``.  A support set S of qubit positions that may differ between
    branches is tracked so that nnz <= 2**|S| <= 2**cap_bits; a draw that
    would grow |S| past the cap is redrawn."""
    rng = _rng(seed)
    regs = [("a", 7), ("b", 7), ("anc", 6)]
    base = [0, 7, 14]                      # flat qubit index of each register
    S: set = set()
    ops = []

    def flat(r, q):
        return base[r] + q

    def unflat(f):
        r = 0 if f < 7 else (1 if f < 14 else 2)
        return r, f - base[r]

    tries = 0
    while len(ops) < nops:
        tries += 1
        if tries > 100000:
            raise RuntimeError("generator could not satisfy the support cap")
        kind = int(rng.integers(0, 5))
        if kind == 0:                                   # H on k qubits of a
            k = int(rng.integers(1, 6))
            qs = rng.choice(7, size=k, replace=False)
            newS = S | {flat(0, int(q)) for q in qs}
            if len(newS) > cap_bits:
                continue
            qmask = 0
            for q in qs:
                qmask |= 1 << int(q)
            ops.append(make_op("H", 0, qmask=qmask))
            S = newS
        elif kind in (1, 2):                            # CNOT / Toffoli
            nq = 2 if kind == 1 else 3
            fs = [int(f) for f in rng.choice(20, size=nq, replace=False)]
            tgt, ctl = fs[0], fs[1:]
            newS = set(S)
            if any(c in S for c in ctl):
                newS.add(tgt)
            if len(newS) > cap_bits:
                continue
            tr, tq = unflat(tgt)
            ctls = [(*unflat(c), 1) for c in ctl]
            ops.append(make_op("X", tr, qmask=1 << tq, ctls=ctls))
            S = newS
        elif kind == 3:                                 # b += a mod 2^7
            pos = [f - base[0] for f in S if f < 7] + [f - base[1] for f in S if 7 <= f < 14]
            newS = set(S)
            if pos:
                lo = min(pos)
                newS |= {flat(1, j) for j in range(lo, 7)}
            if len(newS) > cap_bits:
                continue
            ops.append(make_op("ADD", 1, reg2=0))
            S = newS
        else:                                           # CRy on anc, ctl in a
            tq = int(rng.integers(0, 6))
            cq = int(rng.integers(0, 7))
            theta = float(rng.uniform(0.0, 2.0 * np.pi))
            newS = S | {flat(2, tq)}
            if len(newS) > cap_bits:
                continue
            ops.append(make_op("RY", 2, qmask=1 << tq, theta=theta, ctls=[(0, cq, 1)]))
            S = newS
    return Circuit(regs=regs, ops=ops_array(ops), eps=1e-14, cap_bits=cap_bits,
                   name=f"c1-seed{seed}")


# ---------------------------------------------------------------------------
# C2-form: a, b, c (32 qubits each) + flag; H on 20 qubits of a, then 1000 ops
# ---------------------------------------------------------------------------
def c2_circuit(seed, nops: int = 1000, n_ry: int = 10, h_qubits: int = 20) -> Circuit:
    """Arithmetic-heavy sparse circuit.  Prelude: one H on ``h_qubits`` seeded
    qubits of ``a``.  Then ``nops`` ops of which ``n_ry`` are Ry on the 1-qubit
    ``flag`` at seeded distinct positions; the rest are uniform over ADD, SUB
    (distinct pair of a/b/c), MULC (odd 32-bit constant), XOR (register or
    constant, 50/50), CNOT and Toffoli on distinct qubits of a/b/c.  The flag is
    never a control or operand, so nnz is 2**h_qubits, then twice that after
    the first Ry."""
    rng = _rng(seed)
    regs = [("a", 32), ("b", 32), ("c", 32), ("flag", 1)]
    qs = rng.choice(32, size=h_qubits, replace=False)
    hmask = 0
    for q in qs:
        hmask |= 1 << int(q)
    ops = [make_op("H", 0, qmask=hmask)]
    ry_pos = set(int(p) for p in rng.choice(nops, size=n_ry, replace=False))
    for i in range(nops):
        if i in ry_pos:
            theta = float(rng.uniform(0.0, 2.0 * np.pi))
            ops.append(make_op("RY", 3, qmask=1, theta=theta))
            continue
        kind = int(rng.integers(0, 6))
        if kind in (0, 1):
            d, s = (int(x) for x in rng.choice(3, size=2, replace=False))
            ops.append(make_op("ADD" if kind == 0 else "SUB", d, reg2=s))
        elif kind == 2:
            d = int(rng.integers(0, 3))
            c = int(rng.integers(0, 2 ** 32, dtype=np.uint64)) | 1
            ops.append(make_op("MULC", d, imm=c))
        elif kind == 3:
            d = int(rng.integers(0, 3))
            if rng.integers(0, 2) == 0:
                s = int(rng.choice([r for r in range(3) if r != d]))
                ops.append(make_op("XOR", d, reg2=s))
            else:
                c = int(rng.integers(0, 2 ** 32, dtype=np.uint64))
                ops.append(make_op("XORC", d, imm=c))
        else:
            nq = 2 if kind == 4 else 3
            fs = [int(f) for f in rng.choice(96, size=nq, replace=False)]
            tr, tq = divmod(fs[0], 32)
            ctls = [(f // 32, f % 32, 1) for f in fs[1:]]
            ops.append(make_op("X", tr, qmask=1 << tq, ctls=ctls))
    return Circuit(regs=regs, ops=ops_array(ops), eps=1e-14, cap_bits=h_qubits + 1,
                   name=f"c2-seed{seed}")


# ---------------------------------------------------------------------------
# C3: many C1-form instances with log-uniform caps and uneven lengths
# ---------------------------------------------------------------------------
def c2_rot_circuit(seed, nops: int = 1000, n_ry: int = 10, h_qubits: int = 20) -> Circuit:
    """The arithmetic-heavy circuit with each Ry on the flag replaced by a
    rotation by a seeded Haar-random 2x2 unitary (complex amplitudes)."""
    c = c2_circuit(seed, nops=nops, n_ry=n_ry, h_qubits=h_qubits)
    rng = _rng(np.random.SeedSequence([int(seed), 7]))
    ops = c.ops.copy()
    mats = []
    for i in range(len(ops)):
        if KINDS[int(ops[i]["kind"])] == "RY":
            ops[i]["kind"] = KIND["ROT"]
            ops[i]["table"] = len(mats)
            ops[i]["theta"] = 0.0
            mats.append(random_unitary(rng))
    c.ops = ops
    c.matrices = mats
    c.name = f"c2rot-seed{seed}"
    return c


def c3_batch(seed, ninst: int = 1024, lo_bits: float = 6.0, hi_bits: float = 18.0,
             len_lo: int = 200, len_hi: int = 1000) -> List[Circuit]:
    ss = np.random.SeedSequence(int(seed))
    rng = _rng(ss)
    u = rng.uniform(lo_bits, hi_bits, size=ninst)
    lens = rng.integers(len_lo, len_hi + 1, size=ninst)
    out = []
    for i, child in enumerate(ss.spawn(ninst)):
        c = c1_circuit(child, nops=int(lens[i]), cap_bits=int(np.floor(u[i])))
        c.name = f"c3-seed{seed}-inst{i}"
        out.append(c)
    return out


# ---------------------------------------------------------------------------
# C4: QRAM linear-solver walk batched over right-hand sides
# ---------------------------------------------------------------------------
def c4_matrix(seed, n: int = 1024, nnz_row: int = 8) -> np.ndarray:
    """Random sparse matrix, ``nnz_row`` distinct uniform columns per row,
    N(0,1) values, scaled to spectral norm 1 (dense float64, for the table)."""
    rng = _rng(seed)
    A = np.zeros((n, n))
    for r in range(n):
        cols = rng.choice(n, size=nnz_row, replace=False)
        A[r, cols] = rng.standard_normal(nnz_row)
    A /= np.linalg.norm(A, 2)
    return A


def c4_table(A: np.ndarray, nnz_row: int = 8) -> Tuple[np.ndarray, int]:
    """QRAM words at address row*nnz_row + slot: column index in bits 0..15,
    16-bit two's-complement angle code q16 in bits 16..31, where
    q16 = round-half-even(theta/pi * 2^15) clamped, theta = 2*arcsin(A_rc)
    (the stored rotation angle that loads A_rc as an amplitude)."""
    n = A.shape[0]
    words = np.zeros(n * nnz_row, dtype=np.uint64)
    for r in range(n):
        cols = np.nonzero(A[r])[0]
        for s, c in enumerate(cols):
            theta = 2.0 * np.arcsin(np.clip(A[r, c], -1.0, 1.0))
            q = int(np.round(theta / np.pi * 2 ** 15))      # numpy rounds half to even
            q = max(-2 ** 15, min(2 ** 15 - 1, q))
            words[r * nnz_row + s] = np.uint64(c | ((q & 0xFFFF) << 16))
    return words, int(np.log2(n * nnz_row))


def c4_batch(seed, nrhs: int = 64, steps: int = 200, n: int = 1024, nnz_row: int = 8,
             A: Optional[np.ndarray] = None) -> List[Circuit]:
    """Registers (creation order) data:32, addr:13 (row high, slot low), anc:1.
    Every instance shares one table; instance r starts from a normalised
    complex Gaussian right-hand side on the row field (slot 0, data 0, anc 0).
    Prelude: H on the slot qubits.  Each step: QRAM_LOAD(addr -> data); 16 Ry
    on anc controlled by data bit 16+k with angle pi*2^(k-15) (k<15) and -pi
    (k=15), i.e. Ry(pi*q16/2^15) in total; QRAM_UNLOAD; REFLECT0(anc)."""
    rng = _rng(seed)
    if A is None:
        A = c4_matrix(seed, n, nnz_row)
    words, abits = c4_table(A, nnz_row)
    slot_bits = int(np.log2(nnz_row))
    row_bits = int(np.log2(n))
    regs = [("data", 32), ("addr", abits), ("anc", 1)]
    table = Table(values=words, addr_bits=abits, word_bits=32)
    ops = [make_op("H", 1, qmask=(1 << slot_bits) - 1)]
    for _ in range(steps):
        ops.append(make_op("QRAM_LOAD", 0, reg2=1, table=0))
        for k in range(16):
            ang = np.pi * 2.0 ** (k - 15) if k < 15 else -np.pi
            ops.append(make_op("RY", 2, qmask=1, theta=float(ang), ctls=[(0, 16 + k, 1)]))
        ops.append(make_op("QRAM_UNLOAD", 0, reg2=1, table=0))
        ops.append(make_op("REFLECT0", 2))
    ops = ops_array(ops)
    out = []
    for r in range(nrhs):
        b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
        b /= np.linalg.norm(b)
        vals = np.zeros((n, 3), dtype=np.uint64)
        vals[:, 1] = (np.arange(n, dtype=np.uint64) << np.uint64(slot_bits))
        out.append(Circuit(regs=regs, ops=ops, eps=1e-14, tables=[table],
                           init_values=vals, init_amps=b.astype(np.complex128),
                           cap_bits=row_bits + slot_bits + 1, name=f"c4-seed{seed}-rhs{r}"))
    return out


# ---------------------------------------------------------------------------
# Small and structural circuits for pins and edge cases
# ---------------------------------------------------------------------------
def random_small_circuit(seed, widths=(4, 3, 3, 2), nops: int = 60,
                         kinds: Sequence[str] = BASE_KINDS, max_h: int = 3,
                         eps: float = 1e-14, with_init: bool = False) -> Circuit:
    """Every op kind on a few small registers (<= 20 qubits in total), random
    controls (0-3, on qubits outside the destination register) and a random
    QRAM table; ``with_init`` starts from a random sparse superposition."""
    rng = _rng(seed)
    regs = [(f"r{i}", int(w)) for i, w in enumerate(widths)]
    nr = len(regs)
    tables = []
    # a table addressed by the smallest register, words as wide as the widest
    amin = int(np.argmin(widths))
    dmax = int(np.argmax(widths))
    ab, wb = int(widths[amin]), int(widths[dmax])
    tables.append(Table(values=rng.integers(0, 2 ** wb, size=2 ** ab, dtype=np.uint64),
                        addr_bits=ab, word_bits=wb))
    matrices = []
    if any(k in kinds for k in ("ROT",)):
        # a general unitary, a diagonal one and an anti-diagonal one
        matrices = [random_unitary(rng), random_unitary(rng, "diag"), random_unitary(rng, "anti")]
    ops = []
    while len(ops) < nops:
        kind = str(rng.choice(list(kinds)))
        r = int(rng.integers(0, nr))
        w = int(widths[r])
        others = [x for x in range(nr) if x != r]
        nctl = int(rng.integers(0, 4))
        ctl_pool = [(x, q) for x in range(nr) for q in range(widths[x])]
        if kind in ("ADD", "SUB", "MULC", "XOR", "XORC", "QRAM_LOAD", "QRAM_UNLOAD", "REFLECT0", "ADDC"):
            ctl_pool = [(x, q) for (x, q) in ctl_pool if x != r]
        qmask = 0
        reg3 = reg4 = 0
        table = 0
        if kind in ("X", "Y", "Z", "S", "SDG", "T", "TDG", "PHASE"):
            k = int(rng.integers(1, w + 1))
            for q in rng.choice(w, size=k, replace=False):
                qmask |= 1 << int(q)
        elif kind == "ROT":
            qmask = 1 << int(rng.integers(0, w))
            table = int(rng.integers(0, len(matrices)))
        elif kind == "MUL":
            if nr < 2:
                continue
            reg2, reg3 = (int(x) for x in rng.choice(others, size=2, replace=True))
            ctl_pool = [(x, q) for (x, q) in ctl_pool if x != r]
        elif kind == "DIV":
            if nr < 4:
                continue
            r, r4, reg2, reg3 = (int(x) for x in rng.choice(nr, size=4, replace=False))
            w = int(widths[r])
            reg4 = r4
            ctl_pool = [(x, q) for x in range(nr) for q in range(widths[x]) if x not in (r, r4)]
        elif kind == "H":
            k = int(rng.integers(1, min(max_h, w) + 1))
            for q in rng.choice(w, size=k, replace=False):
                qmask |= 1 << int(q)
        elif kind == "RY":
            qmask = 1 << int(rng.integers(0, w))
        if kind in ("X", "H", "RY", "Y", "Z", "S", "SDG", "T", "TDG", "PHASE", "ROT"):
            ctl_pool = [(x, q) for (x, q) in ctl_pool if not (x == r and (qmask >> q) & 1)]
        if kind not in ("MUL", "DIV"):
            reg2 = 0
        if kind in ("ADD", "SUB", "XOR"):
            reg2 = int(rng.choice(others))
            ctl_pool = [(x, q) for (x, q) in ctl_pool]
        if kind in ("QRAM_LOAD", "QRAM_UNLOAD"):
            if r == amin or widths[r] != wb:
                # data register must be as wide as the table words
                cands = [x for x in range(nr) if x != amin and widths[x] == wb]
                if not cands:
                    continue
                r = int(rng.choice(cands))
                ctl_pool = [(x, q) for x in range(nr) for q in range(widths[x]) if x != r]
            reg2 = amin
        nctl = min(nctl, len(ctl_pool))
        picks = rng.choice(len(ctl_pool), size=nctl, replace=False) if nctl else []
        ctls = [(ctl_pool[int(i)][0], ctl_pool[int(i)][1], int(rng.integers(0, 2))) for i in picks]
        imm = 0
        if kind == "MULC":
            imm = int(rng.integers(0, 2 ** w)) | 1
        elif kind in ("XORC", "ADDC"):
            imm = int(rng.integers(0, 2 ** w))
        theta = float(rng.uniform(0, 2 * np.pi)) if kind in ("RY", "PHASE") else 0.0
        ops.append(make_op(kind, r, qmask=qmask, reg2=reg2, table=table, imm=imm,
                           theta=theta, ctls=ctls, reg3=reg3, reg4=reg4))
    init_values = init_amps = None
    if with_init:
        n0 = int(rng.integers(1, 40))
        total = sum(widths)
        flat = rng.choice(2 ** total, size=n0, replace=False)
        init_values = np.zeros((n0, nr), dtype=np.uint64)
        sh = 0
        for j, w in enumerate(widths):
            init_values[:, j] = (flat >> sh) & ((1 << w) - 1)
            sh += w
        a = rng.standard_normal(n0) + 1j * rng.standard_normal(n0)
        init_amps = (a / np.linalg.norm(a)).astype(np.complex128)
    return Circuit(regs=regs, ops=ops_array(ops), eps=eps, tables=tables,
                   init_values=init_values, init_amps=init_amps, name=f"small-seed{seed}",
                   matrices=matrices)


def random_unitary(rng, form: str = "general") -> np.ndarray:
    """A seeded 2x2 unitary: Haar-random (QR of a complex Gaussian matrix,
    phases fixed by the diagonal of R), or diagonal / anti-diagonal with
    random phases."""
    if form == "diag":
        ph = rng.uniform(0, 2 * np.pi, size=2)
        return np.diag(np.exp(1j * ph)).astype(np.complex128)
    if form == "anti":
        ph = rng.uniform(0, 2 * np.pi, size=2)
        return np.array([[0, np.exp(1j * ph[0])], [np.exp(1j * ph[1]), 0]], dtype=np.complex128)
    z = rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2))
    q, rr = np.linalg.qr(z)
    d = np.diag(rr)
    return (q * (d / np.abs(d))).astype(np.complex128)


def qft_circuit(nqubits: int, x: int, swaps: bool = False) -> Circuit:
    """Textbook quantum Fourier transform of the basis state |x> on one
    register of ``nqubits`` (<= 64) qubits: X on the set bits of x, then for
    j = n-1 down to 0: H on qubit j and, for k = j-1 down to 0, the phase gate
    diag(1, e^{i pi / 2^(j-k)}) on qubit j controlled by qubit k.  Without the
    final swaps the output register holds the transform in bit-reversed
    order; with ``swaps`` each pair (q, n-1-q) is exchanged by three CNOTs.
    Reaches 2^n branches (the qft row of the paper's Table 1 has 29 qubits)."""
    ops = []
    if x:
        ops.append(make_op("X", 0, qmask=int(x)))
    for j in range(nqubits - 1, -1, -1):
        ops.append(make_op("H", 0, qmask=1 << j))
        for k in range(j - 1, -1, -1):
            ops.append(make_op("PHASE", 0, qmask=1 << j, theta=float(np.pi / 2 ** (j - k)), ctls=[(0, k, 1)]))
    if swaps:
        for q in range(nqubits // 2):
            a, b = q, nqubits - 1 - q
            ops += [make_op("X", 0, qmask=1 << b, ctls=[(0, a, 1)]),
                    make_op("X", 0, qmask=1 << a, ctls=[(0, b, 1)]),
                    make_op("X", 0, qmask=1 << b, ctls=[(0, a, 1)])]
    return Circuit(regs=[("q", nqubits)], ops=ops_array(ops), eps=1e-14, cap_bits=nqubits,
                   name=f"qft{nqubits}-x{x}")


def ghz_circuit(nqubits: int) -> Circuit:
    """Textbook GHZ construction: H on qubit 0, then a CNOT chain; registers of
    at most 64 qubits."""
    widths = []
    left = nqubits
    while left > 0:
        widths.append(min(64, left))
        left -= widths[-1]
    regs = [(f"g{i}", w) for i, w in enumerate(widths)]
    flat = [(r, q) for r, w in enumerate(widths) for q in range(w)]
    ops = [make_op("H", 0, qmask=1)]
    for i in range(1, nqubits):
        cr, cq = flat[i - 1]
        tr, tq = flat[i]
        ops.append(make_op("X", tr, qmask=1 << tq, ctls=[(cr, cq, 1)]))
    return Circuit(regs=regs, ops=ops_array(ops), name=f"ghz{nqubits}")


def qram_circuit(seed, addr_bits: int, word_bits: int, superpose: bool = True) -> Circuit:
    """QRAM load on a uniform superposition of addresses (H on every address
    qubit), or on one random address when ``superpose`` is False."""
    rng = _rng(seed)
    values = rng.integers(0, 2 ** word_bits, size=2 ** addr_bits, dtype=np.uint64)
    regs = [("addr", addr_bits), ("data", word_bits)]
    ops = []
    if superpose:
        ops.append(make_op("H", 0, qmask=(1 << addr_bits) - 1))
    else:
        a = int(rng.integers(0, 2 ** addr_bits))
        m = 0
        for q in range(addr_bits):
            if (a >> q) & 1:
                m |= 1 << q
        if m:
            ops.append(make_op("X", 0, qmask=m))
    ops.append(make_op("QRAM_LOAD", 1, reg2=0, table=0))
    return Circuit(regs=regs, ops=ops_array(ops),
                   tables=[Table(values=values, addr_bits=addr_bits, word_bits=word_bits)],
                   name=f"qram{addr_bits}x{word_bits}")


def swap_test_circuit(n: int) -> Circuit:
    """Swap-test form on 2n + 1 qubits: H on every qubit of two n-qubit
    registers x and y (2^(2n) branches), then the textbook swap test: H on the
    ancilla, a controlled swap of x_i and y_i for every i (CNOT, Toffoli, CNOT),
    H on the ancilla.  The peak is 2^(2n+1) branches; x and y being symmetric,
    every ancilla-1 amplitude cancels exactly, leaving 2^(2n) branches."""
    regs = [("x", n), ("y", n), ("anc", 1)]
    full = (1 << n) - 1
    ops = [make_op("H", 0, qmask=full), make_op("H", 1, qmask=full), make_op("H", 2, qmask=1)]
    for i in range(n):
        ops.append(make_op("X", 0, qmask=1 << i, ctls=[(1, i, 1)]))
        ops.append(make_op("X", 1, qmask=1 << i, ctls=[(2, 0, 1), (0, i, 1)]))
        ops.append(make_op("X", 0, qmask=1 << i, ctls=[(1, i, 1)]))
    ops.append(make_op("H", 2, qmask=1))
    return Circuit(regs=regs, ops=ops_array(ops), name=f"swap_test{2 * n + 1}")


# ---------------------------------------------------------------------------
# C5: a Poisson request stream mixing the C1..C4 forms
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class TraceItem:
    arrival: float
    kind: str                     # "c1" | "c2" | "c3" | "c4"
    circuits: List[Circuit]       # one circuit, or C4-form right-hand sides sharing one op list
    peak: int                     # the generator's bound on the peak entry count


def c5_trace(seed, rate: float = 200.0, duration: float = 30.0, lo_bits: float = 8.0,
             hi_bits: float = 24.0, c4_steps: int = 200, c4_matrix_n: int = 1024,
             max_requests: Optional[int] = None) -> List[TraceItem]:
    """Poisson arrivals at `rate` per second for `duration` seconds.  Kind is
    uniform over the four forms; the target peak is P = 2^u, u ~ U[lo, hi]:
    C1/C3 forms (one C1-form circuit) need P <= 2^18, else the kind is redrawn
    among C2/C4; a C2-form request runs H on log2(P) - 1 qubits of a; a
    C4-form request carries max(1, P / 2^14) right-hand sides."""
    rng = _rng(seed)
    t = 0.0
    items: List[TraceItem] = []
    A = None
    words = None
    k = 0
    while True:
        t += float(rng.exponential(1.0 / rate))
        if t > duration or (max_requests is not None and len(items) >= max_requests):
            break
        kind = ("c1", "c2", "c3", "c4")[int(rng.integers(0, 4))]
        u = float(rng.uniform(lo_bits, hi_bits))
        if kind in ("c1", "c3") and u > 18.0:
            kind = ("c2", "c4")[int(rng.integers(0, 2))]
        sub = int(rng.integers(0, 2 ** 31))
        if kind in ("c1", "c3"):
            cb = max(2, int(np.floor(u)))
            circs = [c1_circuit(sub, nops=300, cap_bits=cb)]
            peak = 2 ** cb
        elif kind == "c2":
            h = max(1, int(np.floor(u)) - 1)
            circs = [c2_circuit(sub, nops=1000, n_ry=10, h_qubits=h)]
            peak = 2 ** (h + 1)
        else:
            if A is None:
                A = c4_matrix(seed, n=c4_matrix_n)
            nrhs = max(1, int(2 ** np.floor(u)) // (c4_matrix_n * 16))
            circs = c4_batch(sub, nrhs=nrhs, steps=c4_steps, n=c4_matrix_n, A=A)
            peak = nrhs * c4_matrix_n * 16
        items.append(TraceItem(arrival=t, kind=kind, circuits=circs, peak=peak))
        k += 1
    return items
