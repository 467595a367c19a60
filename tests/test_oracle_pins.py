"""Pins for the CPU oracle against things other than itself.

* a dense brute-force state vector (oracle/dense.py) on random small circuits
  with every op kind and on full C1-form circuits (20 qubits);
* invariants fixed by the mathematics (unitarity, permutation ops preserve nnz
  and the amplitude multiset, H.H = I, QRAM load then unload = I, ADD then SUB,
  MULC by c then by c^-1, XOR twice, Ry(t) Ry(-t));
* closed forms (QRAM on a uniform address superposition, GHZ, H^k |0>, the
  C2-form trajectory structure, the C4-form walk as a 2x2 matrix power);
* branch counts printed in the paper's Table 1 (tests/golden).
"""
import json
import os

import numpy as np
import pytest

import workloads as wl
from oracle.dense import DenseState
from oracle.oracle import OracleState, run_circuit

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
C = 0.70710678118654752440


def _sorted_entries(vals, amps):
    order = np.lexsort(vals.T[::-1]) if len(vals) else np.arange(0)
    return vals[order], amps[order]


def _oracle_vs_dense(c, tol=1e-13):
    st, _, _ = run_circuit(c)
    _, v, a = st.export()
    d = DenseState.from_circuit(c)
    d.apply(c.ops)
    dv, da = d.entries()
    v, a = _sorted_entries(v, a)
    dv, da = _sorted_entries(dv, da)
    assert v.shape == dv.shape, (v.shape, dv.shape)
    assert np.array_equal(v, dv)
    if len(a):
        assert np.max(np.abs(a - da)) <= tol
    return st


@pytest.mark.parametrize("seed", range(16))
def test_oracle_matches_dense_small(seed):
    c = wl.random_small_circuit(seed, with_init=bool(seed % 2), eps=(0.0 if seed % 4 == 3 else 1e-14))
    _oracle_vs_dense(c)


@pytest.mark.parametrize("seed", [0, 1])
def test_oracle_matches_dense_c1(seed):
    c = wl.c1_circuit(seed)
    st = _oracle_vs_dense(c)
    assert st.peak <= 2 ** 14


def test_generator_is_deterministic():
    a = wl.c1_circuit(7).ops.tobytes()
    b = wl.c1_circuit(7).ops.tobytes()
    assert a == b
    assert wl.c2_circuit(3).ops.tobytes() == wl.c2_circuit(3).ops.tobytes()


def test_packing_rule():
    # first fit in creation order, never straddling a 64-bit word
    st = OracleState([("a", 32), ("b", 32), ("c", 32), ("flag", 1)])
    assert [st.layout(r) for r in range(4)] == [(0, 0), (0, 32), (1, 0), (1, 32)]
    st = OracleState([("x", 40), ("y", 30), ("z", 20)])
    assert [st.layout(r) for r in range(3)] == [(0, 0), (1, 0), (0, 40)]


def _norm2(amps):
    return float(np.sum(amps.real ** 2 + amps.imag ** 2))


@pytest.mark.parametrize("seed", range(6))
def test_norm_is_preserved(seed):
    c = wl.random_small_circuit(seed, eps=0.0, with_init=True)
    st, _, _ = run_circuit(c)
    _, _, a = st.export()
    assert abs(_norm2(a) - 1.0) < 1e-12


@pytest.mark.parametrize("seed", range(6))
def test_permutation_ops_keep_amplitude_multiset(seed):
    kinds = ("X", "ADD", "SUB", "MULC", "XOR", "XORC", "QRAM_LOAD", "QRAM_UNLOAD")
    c = wl.random_small_circuit(seed, kinds=kinds, nops=80, with_init=True)
    st0 = OracleState.from_circuit(c)
    _, _, a0 = st0.export()
    st, _, _ = run_circuit(c)
    _, _, a1 = st.export()
    assert st.nnz == st0.nnz
    bits0 = sorted(map(tuple, a0.view(np.uint64).reshape(-1, 2).tolist()))
    bits1 = sorted(map(tuple, a1.view(np.uint64).reshape(-1, 2).tolist()))
    assert bits0 == bits1


def _start(seed, widths=(4, 3, 3, 2)):
    return wl.random_small_circuit(seed, widths=widths, nops=1, with_init=True)


@pytest.mark.parametrize("seed", range(5))
def test_h_h_is_identity(seed):
    c = _start(seed)
    ops = wl.ops_array([wl.make_op("H", 0, qmask=0b1011), wl.make_op("H", 0, qmask=0b1011)])
    st = OracleState(c.regs, 1e-14, c.tables, c.init_values, c.init_amps)
    k0, _, a0 = st.export()
    st.apply(ops)
    k1, _, a1 = st.export()
    assert np.array_equal(k0, k1)
    assert np.max(np.abs(a0 - a1)) < 4 * np.finfo(float).eps


@pytest.mark.parametrize("seed", range(5))
def test_inverse_pairs_are_exact_identities(seed):
    c = _start(seed)
    inv7 = pow(7, -1, 16)
    ops = wl.ops_array([
        wl.make_op("QRAM_LOAD", 1, reg2=3, table=0),
        wl.make_op("QRAM_UNLOAD", 1, reg2=3, table=0),
        wl.make_op("ADD", 0, reg2=2, ctls=[(1, 0, 1)]),
        wl.make_op("SUB", 0, reg2=2, ctls=[(1, 0, 1)]),
        wl.make_op("MULC", 0, imm=7),
        wl.make_op("MULC", 0, imm=inv7),
        wl.make_op("XOR", 2, reg2=0),
        wl.make_op("XOR", 2, reg2=0),
    ])
    tab = wl.Table(values=np.array([5, 1, 7, 2], dtype=np.uint64), addr_bits=2, word_bits=3)
    st = OracleState(c.regs, 1e-14, [tab], c.init_values, c.init_amps)
    k0, _, a0 = st.export()
    st.apply(ops)
    k1, _, a1 = st.export()
    assert np.array_equal(k0, k1)
    assert np.array_equal(a0.view(np.uint64), a1.view(np.uint64))


def test_ry_then_inverse():
    c = _start(3)
    st = OracleState(c.regs, 1e-14, c.tables, c.init_values, c.init_amps)
    k0, _, a0 = st.export()
    st.apply(wl.ops_array([wl.make_op("RY", 1, qmask=2, theta=1.234),
                           wl.make_op("RY", 1, qmask=2, theta=-1.234)]))
    k1, _, a1 = st.export()
    assert np.array_equal(k0, k1)
    assert np.max(np.abs(a0 - a1)) < 1e-15


def test_ry_pi_on_zero_gives_one_key():
    st = OracleState([("q", 1)])
    st.apply(wl.ops_array([wl.make_op("RY", 0, qmask=1, theta=np.pi)]))
    _, v, a = st.export()
    assert v.tolist() == [[1]]
    assert a[0] == 1.0 + 0j


def test_ry_sign_convention():
    # Ry(t)|0> = cos(t/2)|0> + sin(t/2)|1>,  Ry(t)|1> = -sin(t/2)|0> + cos(t/2)|1>
    t = 0.7
    st = OracleState([("q", 1)])
    st.apply(wl.ops_array([wl.make_op("RY", 0, qmask=1, theta=t)]))
    _, v, a = st.export()
    assert v[:, 0].tolist() == [0, 1]
    assert a[0] == np.cos(t / 2) and a[1] == np.sin(t / 2)
    st = OracleState([("q", 1)], init_values=np.array([[1]], dtype=np.uint64),
                     init_amps=np.array([1.0 + 0j]))
    st.apply(wl.ops_array([wl.make_op("RY", 0, qmask=1, theta=t)]))
    _, v, a = st.export()
    assert a[0] == -np.sin(t / 2) and a[1] == np.cos(t / 2)


def test_reflection_phases():
    # R = i(2|0><0| - I): +i on anc = 0, -i otherwise
    st = OracleState([("anc", 2), ("x", 2)], init_values=np.array([[0, 1], [2, 1]], dtype=np.uint64),
                     init_amps=np.array([0.6 + 0j, 0.0 + 0.8j]))
    st.apply(wl.ops_array([wl.make_op("REFLECT0", 0)]))
    _, v, a = st.export()
    assert v.tolist() == [[0, 1], [2, 1]]
    assert a[0] == 0.6j and a[1] == 0.8 + 0j


@pytest.mark.parametrize("k", [1, 3, 5, 8])
def test_h_power_on_zero(k):
    st = OracleState([("a", 10)])
    st.apply(wl.ops_array([wl.make_op("H", 0, qmask=(1 << k) - 1)]))
    _, v, a = st.export()
    assert v[:, 0].tolist() == list(range(2 ** k))
    expect = 1.0
    for _ in range(k):
        expect = C * expect
    assert np.all(a == expect)


@pytest.mark.parametrize("addr_bits,word_bits", [(4, 6), (10, 10), (12, 32)])
def test_qram_closed_form(addr_bits, word_bits):
    c = wl.qram_circuit(addr_bits, addr_bits, word_bits)
    st, _, _ = run_circuit(c)
    _, v, a = st.export()
    d = c.tables[0].values
    got = {int(x): int(y) for x, y in v}
    assert got == {i: int(d[i]) for i in range(2 ** addr_bits)}
    expect = 1.0
    for _ in range(addr_bits):
        expect = C * expect
    assert np.all(a == expect)


def test_paper_branch_counts():
    g = json.load(open(os.path.join(GOLDEN, "paper_branch_counts.json")))
    for nq, branches in g["ghz"]:
        st, _, _ = run_circuit(wl.ghz_circuit(nq))
        _, v, a = st.export()
        assert st.nnz == branches
        assert np.all(a == C)
        ones = [(1 << w) - 1 for _, w in wl.ghz_circuit(nq).regs]
        assert v.tolist() == [[0] * len(ones), ones]
    for nq, branches in g["qram"]:
        c = wl.qram_circuit(1, nq // 2, nq - nq // 2, superpose=False)
        st, _, _ = run_circuit(c)
        assert st.nnz == branches


def test_c2_form_closed_form():
    """Keys are the classical trajectories of the initial values of a through the
    composed permutations (replayed here with vectorised numpy), times flag in
    {0,1}; amplitudes are c^h * (Ry(t_m)...Ry(t_1)|0>)_flag."""
    h = 6
    c = wl.c2_circuit(11, nops=150, n_ry=4, h_qubits=h)
    st, _, _ = run_circuit(c)
    _, v, a = st.export()
    hmask = int(c.ops[0]["qmask"])
    qs = [q for q in range(32) if (hmask >> q) & 1]
    starts = np.array([sum(((i >> j) & 1) << q for j, q in enumerate(qs)) for i in range(2 ** h)],
                      dtype=np.uint64)
    regs = np.zeros((2 ** h, 3), dtype=np.uint64)
    regs[:, 0] = starts
    M = np.uint64(0xFFFFFFFF)
    vec = np.array([1.0, 0.0])
    for op in c.ops[1:]:
        kind = wl.KINDS[int(op["kind"])]
        d = int(op["reg"])
        if kind == "RY":
            t = float(op["theta"]) / 2
            vec = np.array([[np.cos(t), -np.sin(t)], [np.sin(t), np.cos(t)]]) @ vec
            continue
        s = int(op["reg2"])
        if kind == "ADD":
            regs[:, d] = (regs[:, d] + regs[:, s]) & M
        elif kind == "SUB":
            regs[:, d] = (regs[:, d] - regs[:, s]) & M
        elif kind == "MULC":
            regs[:, d] = (regs[:, d] * np.uint64(op["imm"])) & M
        elif kind == "XOR":
            regs[:, d] ^= regs[:, s]
        elif kind == "XORC":
            regs[:, d] ^= np.uint64(op["imm"])
        elif kind == "X":
            on = np.ones(len(regs), dtype=bool)
            for j in range(int(op["nctl"])):
                on &= ((regs[:, int(op["ctl_reg"][j])] >> np.uint64(op["ctl_qubit"][j])) & np.uint64(1)) == 1
            regs[on, d] ^= np.uint64(op["qmask"])
    expect = {}
    amp0 = 1.0
    for _ in range(h):
        amp0 = C * amp0
    for r in regs:
        for f in (0, 1):
            if abs(vec[f]) >= 1e-14:
                expect[(int(r[0]), int(r[1]), int(r[2]), f)] = amp0 * vec[f]
    got = {tuple(int(x) for x in row): amp for row, amp in zip(v, a)}
    assert set(got) == set(expect)
    for k, amp in got.items():
        assert abs(amp - expect[k]) < 1e-13


def test_c4_form_closed_form():
    """alpha(r, s, anc) = b_r * c^3 * [(R Ry(theta_rs))^T e0]_anc with
    theta_rs = pi*q16/2^15 from the table word (16 controlled Ry whose angles
    add up, then the reflection)."""
    n, steps = 64, 5
    circ = wl.c4_batch(5, nrhs=2, steps=steps, n=n)
    words = circ[0].tables[0].values
    for c in circ[:2]:
        st, _, _ = run_circuit(c)
        _, v, a = st.export()
        b = c.init_amps
        R = np.array([[1j, 0], [0, -1j]])
        got = {tuple(int(x) for x in row): amp for row, amp in zip(v, a)}
        expect = {}
        for r in range(n):
            for s in range(8):
                w = int(words[r * 8 + s])
                q = (w >> 16) & 0xFFFF
                q = q - 65536 if q >= 32768 else q
                t = np.pi * q / 2 ** 15 / 2
                U = R @ np.array([[np.cos(t), -np.sin(t)], [np.sin(t), np.cos(t)]])
                vec = np.linalg.matrix_power(U, steps) @ np.array([1.0, 0.0])
                for anc in (0, 1):
                    amp = b[r] * C * C * C * vec[anc]
                    if abs(amp) >= 1e-14:
                        expect[(0, (r << 3) | s, anc)] = amp
        assert set(got) == set(expect)
        err = max(abs(got[k] - expect[k]) for k in got)
        assert err < 1e-12


@pytest.mark.parametrize("seed", range(4))
def test_measure_matches_dense_marginals(seed):
    c = wl.random_small_circuit(seed, nops=30, with_init=True)
    st, _, _ = run_circuit(c)
    d = DenseState.from_circuit(c)
    d.apply(c.ops)
    dv, da = d.entries()
    reg = seed % len(c.regs)
    p = {}
    for row, amp in zip(dv, da):
        p[int(row[reg])] = p.get(int(row[reg]), 0.0) + abs(amp) ** 2
    keys = sorted(p)
    P = sum(p[k] for k in keys)
    cum = np.cumsum([p[k] for k in keys])
    u = 0.37
    # skip draws that land within 1e-9 of a cumulative boundary
    if np.min(np.abs(cum - u * P)) < 1e-9:
        pytest.skip("draw on a boundary")
    expect_v = keys[int(np.searchsorted(cum, u * P, side="right"))]
    v, prob = st.measure(reg, u)
    assert v == expect_v
    assert abs(prob - p[v] / P) < 1e-12
    _, vals, amps = st.export()
    assert np.all(vals[:, reg] == v)
    assert abs(_norm2(amps) - 1.0) < 1e-12


def test_prune_threshold_is_strict():
    st = OracleState([("q", 2)], eps=0.0,
                     init_values=np.array([[0], [1], [2]], dtype=np.uint64),
                     init_amps=np.array([1e-3 + 0j, 1e-5 + 0j, 0.9 + 0j]))
    st.prune(1e-5)          # |a|^2 == eps^2 is kept
    assert st.nnz == 3
    st.prune(1.0001e-5)
    assert st.nnz == 2


@pytest.mark.parametrize("n", [1, 3])
def test_swap_test_closed_form(n):
    """Swap test on symmetric inputs: the ancilla ends in |0> for every (x, y),
    each with amplitude c^(2n) (2 c^(2n+2) = c^(2n)); the peak is 2^(2n+1)."""
    c = wl.swap_test_circuit(n)
    st, _, _ = run_circuit(c)
    _, v, a = st.export()
    assert st.nnz == 2 ** (2 * n)
    assert st.peak == 2 ** (2 * n + 1)
    assert sorted((int(x), int(y)) for x, y, _ in v) == [(x, y) for x in range(2 ** n) for y in range(2 ** n)]
    assert np.all(v[:, 2] == 0)
    expect = C ** (2 * n)
    assert np.allclose(a, expect, rtol=0, atol=1e-15)
    # dense brute force agrees on the whole state
    d = DenseState.from_circuit(c)
    d.apply(c.ops)
    dv, da = _sorted_entries(*d.entries())
    v, a = _sorted_entries(v, a)
    assert np.array_equal(dv, v)
    assert np.allclose(da, a, rtol=0, atol=1e-15)
