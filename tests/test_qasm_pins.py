"""The OpenQASM 2.0 subset front end (paper_2503_15118_amd/qasm.py) on the
CPU oracle: expression evaluation, gate conventions pinned through identities
with gates whose semantics the oracle pins already (H, X, Z, Ry), controlled
and two-qubit gates, QFT and GHZ texts (including registers longer than 64
qubits), round trip through text, and the oracle against the dense checker
on random programs."""
import numpy as np
import pytest

import workloads as wl
from oracle.dense import DenseState
from oracle.oracle import OracleState
from paper_2503_15118_amd import qasm

C = 0.70710678118654752440


def test_expressions():
    assert qasm._eval_expr("pi/2") == np.pi / 2
    assert qasm._eval_expr("-3*pi/4") == -3 * np.pi / 4
    assert qasm._eval_expr("(1+2)*0.5") == 1.5
    assert qasm._eval_expr("2e-3") == 0.002
    assert qasm._eval_expr("-(pi - 1)/-2") == (np.pi - 1) / 2
    with pytest.raises(ValueError):
        qasm._eval_expr("pi pi")


def _state(seed, n=3):
    rng = np.random.default_rng(seed)
    vals = np.arange(2 ** n, dtype=np.uint64).reshape(-1, 1)
    a = rng.standard_normal(2 ** n) + 1j * rng.standard_normal(2 ** n)
    return vals, a / np.linalg.norm(a)


def _run(text, seed=0, n=3):
    p = qasm.parse(text, eps=0.0)
    vals, a = _state(seed, n)
    st = OracleState(p.circuit.regs, 0.0, init_values=vals, init_amps=a, matrices=p.circuit.matrices)
    st.apply(p.circuit.ops)
    _, v, amp = st.export()
    out = np.zeros(2 ** n, dtype=np.complex128)
    out[v[:, 0].astype(np.int64)] = amp
    return out


def _vec(gates, seed=0, n=3):
    return _run("OPENQASM 2.0;\ninclude \"qelib1.inc\";\nqreg q[%d];\n%s" % (n, gates), seed, n)


@pytest.mark.parametrize("seed", range(3))
def test_single_qubit_conventions(seed):
    t = 0.731
    # u3 and u2 reduce to ry, rx and H; rz is p up to a global phase; sx^2 = X
    assert np.allclose(_vec(f"u3({t},0,0) q[1];", seed), _vec(f"ry({t}) q[1];", seed), atol=1e-15)
    assert np.allclose(_vec(f"u3({t},-pi/2,pi/2) q[1];", seed), _vec(f"rx({t}) q[1];", seed), atol=1e-15)
    assert np.allclose(_vec("u2(0,pi) q[1];", seed), _vec("h q[1];", seed), atol=1e-15)
    assert np.allclose(_vec(f"rz({t}) q[1];", seed), np.exp(-0.5j * t) * _vec(f"p({t}) q[1];", seed), atol=1e-15)
    assert np.allclose(_vec("sx q[1]; sx q[1];", seed), _vec("x q[1];", seed), atol=1e-15)
    assert np.allclose(_vec("sx q[1]; sxdg q[1];", seed), _vec("id q[1];", seed), atol=1e-15)
    assert np.allclose(_vec("u1(pi) q[1];", seed), _vec("z q[1];", seed), atol=1e-15)
    assert np.allclose(_vec("rx(pi) q[1];", seed), -1j * _vec("x q[1];", seed), atol=1e-15)
    assert np.allclose(_vec("h q[1]; z q[1]; h q[1];", seed), _vec("x q[1];", seed), atol=1e-15)
    assert np.allclose(_vec("s q[1]; s q[1];", seed), _vec("z q[1];", seed), atol=1e-15)
    assert np.allclose(_vec("t q[1]; t q[1];", seed), _vec("s q[1];", seed), atol=1e-15)
    assert np.allclose(_vec("y q[1];", seed), 1j * _vec("z q[1]; x q[1];", seed), atol=1e-15)


@pytest.mark.parametrize("seed", range(3))
def test_two_qubit_conventions(seed):
    v0 = _vec("id q[0];", seed)
    # cz and cp are symmetric in their qubits; swap exchanges amplitudes
    assert np.allclose(_vec("cz q[0], q[2];", seed), _vec("cz q[2], q[0];", seed), atol=0)
    assert np.allclose(_vec("cp(0.4) q[0], q[2];", seed), _vec("cp(0.4) q[2], q[0];", seed), atol=1e-16)
    sw = _vec("swap q[0], q[2];", seed)
    perm = [int(format(i, "03b")[::-1], 2) for i in range(8)]   # exchanging bits 0 and 2 = reversing 3 bits
    assert np.array_equal(sw, v0[perm])
    # cx: flips qubit 1 where qubit 0 is 1
    cx = _vec("cx q[0], q[1];", seed)
    idx = [i ^ 2 if i & 1 else i for i in range(8)]
    assert np.array_equal(cx, v0[idx])
    ccx = _vec("ccx q[0], q[1], q[2];", seed)
    idx = [i ^ 4 if (i & 3) == 3 else i for i in range(8)]
    assert np.array_equal(ccx, v0[idx])
    # controlled-U acts as U on the control-1 half only
    cry = _vec("cry(0.9) q[2], q[0];", seed)
    ry = _vec("ry(0.9) q[0];", seed)
    assert np.allclose(cry[4:], ry[4:], atol=1e-16) and np.array_equal(cry[:4], v0[:4])


def test_qft_text_round_trip():
    """The QFT-form circuit written as QASM text and read back gives the same
    state (and the closed form of the transform)."""
    n, x = 7, 83
    c = wl.qft_circuit(n, x, swaps=True)
    p = qasm.parse(qasm.to_qasm(c))
    st = OracleState.from_circuit(p.circuit)
    st.apply(p.circuit.ops)
    _, v, a = st.export()
    expect = np.exp(2j * np.pi * ((x * v[:, 0].astype(np.int64)) % 2 ** n) / 2 ** n) / 2 ** (n / 2)
    assert len(a) == 2 ** n and np.max(np.abs(a - expect)) < 1e-13


def test_ghz_over_long_register():
    """A qreg of 100 qubits splits into registers of 64 and 36; GHZ gives two
    branches of amplitude 1/sqrt 2."""
    n = 100
    text = "OPENQASM 2.0;\nqreg q[%d];\ncreg c[%d];\nh q[0];\n" % (n, n)
    text += "".join(f"cx q[{i}], q[{i + 1}];\n" for i in range(n - 1))
    text += "measure q -> c;\n"
    p = qasm.parse(text)
    assert [w for _, w in p.circuit.regs] == [64, 36]
    assert len(p.measures) == n
    st = OracleState.from_circuit(p.circuit)
    st.apply(p.circuit.ops)
    _, v, a = st.export()
    assert v.tolist() == [[0, 0], [2 ** 64 - 1, 2 ** 36 - 1]]
    assert np.all(a == C)


def random_program(seed, nq=(5, 4), ngates=60):
    """A random program over the supported gates on two qregs."""
    rng = np.random.default_rng(seed)
    names = ["a", "b"]
    qs = [(names[r], i) for r in range(2) for i in range(nq[r])]
    one = ["x", "y", "z", "h", "s", "sdg", "t", "tdg", "sx", "sxdg"]
    par = ["rx", "ry", "rz", "p", "u1"]
    two = ["cx", "cy", "cz", "ch", "swap", "cp", "crz", "cry", "crx"]
    lines = ["OPENQASM 2.0;", 'include "qelib1.inc";'] + [f"qreg {nm}[{w}];" for nm, w in zip(names, nq)]
    for _ in range(ngates):
        k = rng.integers(0, 5)
        pick = [qs[int(i)] for i in rng.choice(len(qs), size=3, replace=False)]
        q = [f"{r}[{i}]" for r, i in pick]
        if k == 0:
            lines.append(f"{rng.choice(one)} {q[0]};")
        elif k == 1:
            lines.append(f"{rng.choice(par)}({rng.uniform(-4, 4)!r}) {q[0]};")
        elif k == 2:
            g = str(rng.choice(two))
            arg = f"({rng.uniform(-4, 4)!r})" if g in ("cp", "crz", "cry", "crx") else ""
            lines.append(f"{g}{arg} {q[0]}, {q[1]};")
        elif k == 3:
            lines.append(f"u3({rng.uniform(0, 3)!r},{rng.uniform(-3, 3)!r},{rng.uniform(-3, 3)!r}) {q[0]};")
        else:
            lines.append(f"ccx {q[0]}, {q[1]}, {q[2]};")
    lines.append("h a;")
    return "\n".join(lines) + "\n"


@pytest.mark.parametrize("seed", range(6))
def test_random_programs_oracle_vs_dense(seed):
    p = qasm.parse(random_program(seed), eps=1e-14)
    c = p.circuit
    st = OracleState.from_circuit(c)
    st.apply(c.ops)
    _, v, a = st.export()
    d = DenseState.from_circuit(c)
    d.apply(c.ops)
    dv, da = d.entries()
    o1, o2 = np.lexsort(v.T[::-1]), np.lexsort(dv.T[::-1])
    assert np.array_equal(v[o1], dv[o2])
    assert np.max(np.abs(a[o1] - da[o2])) < 1e-13


def test_unsupported_statements():
    for bad in ("gate foo a { x a; }", "qreg q[2]; reset q[0];", "qreg q[2]; foo q[0];"):
        with pytest.raises(ValueError):
            qasm.parse("OPENQASM 2.0;\n" + bad)
