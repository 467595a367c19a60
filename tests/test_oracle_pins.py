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


@pytest.mark.parametrize("seed,nops,n_ry,h", [(11, 150, 4, 6), (3, 400, 6, 10), (0, 1000, 10, 8)])
def test_c2_form_closed_form(seed, nops, n_ry, h):
    """Keys are the classical trajectories of the initial values of a through the
    composed permutations (vectorised numpy replay, oracle/closed_forms.py),
    times flag in {0,1}; amplitudes are c^h * (Ry(t_m)...Ry(t_1)|0>)_flag.
    Checked against the map oracle entry by entry."""
    from oracle.closed_forms import c2_closed_form
    from parity import compare_arrays
    c = wl.c2_circuit(seed, nops=nops, n_ry=n_ry, h_qubits=h)
    st, _, _ = run_circuit(c)
    ok, _, oa = st.export()
    ck, ca = c2_closed_form(c)
    s = compare_arrays(ck, ca, ok, oa, c.eps, atol=1e-13)
    assert s["n_gpu"] == s["n_oracle"] == s["shared"] == 2 ** (h + 1)


@pytest.mark.parametrize("seed", [1, 4])
def test_c2_rot_form_closed_form(seed):
    """The same structure with complex rotations on the flag."""
    from oracle.closed_forms import c2_closed_form
    from parity import compare_arrays
    c = wl.c2_rot_circuit(seed, nops=300, n_ry=5, h_qubits=8)
    st, _, _ = run_circuit(c)
    ok, _, oa = st.export()
    ck, ca = c2_closed_form(c)
    s = compare_arrays(ck, ca, ok, oa, c.eps, atol=1e-13)
    assert s["n_gpu"] == s["n_oracle"] == 2 ** 9
    assert np.max(np.abs(oa.imag)) > 0.01


def test_compare_arrays_catches_mistakes():
    """The vectorised comparison flags a missing key, a wrong key word, a
    wrong amplitude and a non-ascending export; band keys may be missing."""
    from parity import compare_arrays
    rng = np.random.default_rng(0)
    w1 = np.sort(rng.choice(1 << 40, size=300, replace=False)).astype(np.uint64)
    keys = np.stack([rng.integers(0, 1 << 62, size=300).astype(np.uint64), w1], axis=1)
    amps = rng.normal(size=300) + 1j * rng.normal(size=300)
    compare_arrays(keys, amps, keys, amps, 1e-14)
    with pytest.raises(AssertionError):
        compare_arrays(keys[1:], amps[1:], keys, amps, 1e-14)
    k2 = keys.copy()
    k2[5, 0] ^= np.uint64(1)
    with pytest.raises(AssertionError):
        compare_arrays(k2, amps, keys, amps, 1e-14)
    a2 = amps.copy()
    a2[7] += 2e-12
    with pytest.raises(AssertionError):
        compare_arrays(keys, a2, keys, amps, 1e-14)
    with pytest.raises(AssertionError):
        compare_arrays(keys[::-1], amps[::-1], keys, amps, 1e-14)
    a3 = amps.copy()
    a3[9] = 1e-10
    compare_arrays(np.delete(keys, 9, 0), np.delete(amps, 9), keys, a3, 1e-14)


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


def test_measure_extreme_draws():
    """u = 0 picks the smallest field value with weight, u just below 1 the
    largest; the probabilities are the marginals."""
    vals = np.array([[1, 0], [3, 1], [3, 2], [6, 3]], dtype=np.uint64)
    amps = np.array([0.5, 0.5j, -0.5, 0.5], dtype=np.complex128)
    for u, expect, p in ((0.0, 1, 0.25), (np.nextafter(1.0, 0.0), 6, 0.25), (0.3, 3, 0.5)):
        st = OracleState([("x", 3), ("y", 2)], 1e-14, init_values=vals, init_amps=amps)
        v, prob = st.measure(0, float(u))
        assert v == expect and prob == p
        _, kv, ka = st.export()
        keep = vals[:, 0] == expect
        assert kv.tolist() == vals[keep].tolist()
        assert np.allclose(ka, amps[keep] / np.sqrt(p), rtol=0, atol=1e-15)


def test_measure_fallback_takes_largest_value():
    """When no running sum exceeds u*P (here P is subnormal, 2e-322, and
    0.99*P rounds back to P) the outcome is the largest field value with
    weight: the fallback branch of the reading."""
    a = 1e-161
    assert a * a > 0 and 0.99 * (a * a + a * a) == a * a + a * a
    vals = np.array([[2], [5]], dtype=np.uint64)
    st = OracleState([("x", 3)], 0.0, init_values=vals, init_amps=np.array([a, a], dtype=np.complex128))
    v, prob = st.measure(0, 0.99)
    assert v == 5 and prob == 0.5


# ---------------------------------------------------------------------------
# The rest of the gate and oracle set: Y, Z, S, T (and inverses), the phase
# gate, a general 2x2 rotation (diagonal, off-diagonal and general matrices),
# add-constant, multiply and divide.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed", range(14))
def test_oracle_matches_dense_all_kinds(seed):
    c = wl.random_small_circuit(seed, kinds=wl.KINDS, nops=70, with_init=bool(seed % 2),
                                eps=(0.0 if seed % 4 == 3 else 1e-14))
    kinds = {wl.KINDS[int(k)] for k in c.ops["kind"]}
    assert len(kinds) >= 12
    _oracle_vs_dense(c)


def _run_ops(c, ops, matrices=()):
    st = OracleState(c.regs, c.eps, c.tables, c.init_values, c.init_amps, matrices)
    st.apply(wl.ops_array(ops))
    return st.export()


@pytest.mark.parametrize("seed", range(4))
def test_phase_gate_identities(seed):
    """Z.Z = I, S.S = Z and S.S^-1 = I bit for bit (factors -1 and +-i are
    exact); T.T = S and T.T^-1 = I within rounding; the phase gate at pi/2
    is S within rounding; Y equals i X Z."""
    c = _start(seed)
    ctl = [(1, 0, 1)]
    k0, _, a0 = _run_ops(c, [])
    kz, _, az = _run_ops(c, [wl.make_op("Z", 0, qmask=0b0110, ctls=ctl)])
    k1, _, a1 = _run_ops(c, [wl.make_op("Z", 0, qmask=0b0110, ctls=ctl)] * 2)
    assert np.array_equal(k0, k1) and np.array_equal(a0.view(np.uint64), a1.view(np.uint64))
    ks, _, as_ = _run_ops(c, [wl.make_op("S", 0, qmask=0b0110, ctls=ctl)] * 2)
    assert np.array_equal(ks, kz) and np.array_equal(np.abs(as_ - az), np.zeros(len(az)))
    k2, _, a2 = _run_ops(c, [wl.make_op("S", 0, qmask=0b1011), wl.make_op("SDG", 0, qmask=0b1011)])
    assert np.array_equal(k2, k0) and np.array_equal(a2.view(np.uint64), a0.view(np.uint64))
    kt, _, at = _run_ops(c, [wl.make_op("T", 0, qmask=0b0110, ctls=ctl)] * 2)
    ks1, _, as1 = _run_ops(c, [wl.make_op("S", 0, qmask=0b0110, ctls=ctl)])
    assert np.array_equal(kt, ks1) and np.max(np.abs(at - as1)) < 1e-15
    k3, _, a3 = _run_ops(c, [wl.make_op("T", 0, qmask=0b1111), wl.make_op("TDG", 0, qmask=0b1111)])
    assert np.array_equal(k3, k0) and np.max(np.abs(a3 - a0)) < 1e-15
    kp, _, ap = _run_ops(c, [wl.make_op("PHASE", 0, qmask=0b0110, theta=np.pi / 2, ctls=ctl)])
    assert np.array_equal(kp, ks1) and np.max(np.abs(ap - as1)) < 1e-15
    ky, vy, ay = _run_ops(c, [wl.make_op("Y", 0, qmask=0b0101, ctls=ctl)])
    kxz, _, axz = _run_ops(c, [wl.make_op("Z", 0, qmask=0b0101, ctls=ctl), wl.make_op("X", 0, qmask=0b0101, ctls=ctl)])
    # on each qubit Y = i X Z: two qubits give i^2 = -1 where the control holds
    assert np.array_equal(ky, kxz)
    on = (vy[:, 1] & 1) == 1
    assert np.max(np.abs(ay - np.where(on, -axz, axz))) < 1e-15


def test_y_on_basis_states():
    # Y|0> = i|1>, Y|1> = -i|0>
    st = OracleState([("q", 1)], init_values=np.array([[0], [1]], dtype=np.uint64),
                     init_amps=np.array([0.6, 0.8], dtype=np.complex128))
    st.apply(wl.ops_array([wl.make_op("Y", 0, qmask=1)]))
    _, v, a = st.export()
    assert v[:, 0].tolist() == [0, 1]
    assert a[0] == -0.8j and a[1] == 0.6j


def test_hzh_is_x_and_hyh_is_minus_y():
    c = _start(2)
    kx, _, ax = _run_ops(c, [wl.make_op("X", 0, qmask=0b0100)])
    kh, _, ah = _run_ops(c, [wl.make_op("H", 0, qmask=0b0100), wl.make_op("Z", 0, qmask=0b0100),
                             wl.make_op("H", 0, qmask=0b0100)])
    assert np.array_equal(kx, kh) and np.max(np.abs(ax - ah)) < 1e-15
    ky, _, ay = _run_ops(c, [wl.make_op("Y", 0, qmask=0b0100)])
    kh, _, ah = _run_ops(c, [wl.make_op("H", 0, qmask=0b0100), wl.make_op("Y", 0, qmask=0b0100),
                             wl.make_op("H", 0, qmask=0b0100)])
    assert np.array_equal(ky, kh) and np.max(np.abs(ay + ah)) < 1e-15


@pytest.mark.parametrize("seed", range(4))
def test_rotation_matrices(seed):
    """ROT by a Haar-random U then by U^dagger is the identity (stray keys
    cancel below eps); ROT by a diagonal or off-diagonal unitary keeps nnz and
    every |a| (one branch per branch); ROT by H's matrix equals the H op."""
    rng = np.random.default_rng(seed)
    c = _start(seed)
    U = wl.random_unitary(rng)
    D = wl.random_unitary(rng, "diag")
    A = wl.random_unitary(rng, "anti")
    Hm = np.array([[C, C], [C, -C]], dtype=np.complex128)
    mats = [U, U.conj().T, D, A, Hm]
    k0, _, a0 = _run_ops(c, [])
    ctl = [(2, 1, 0)]
    k1, _, a1 = _run_ops(c, [wl.make_op("ROT", 0, qmask=4, table=0, ctls=ctl),
                             wl.make_op("ROT", 0, qmask=4, table=1, ctls=ctl)], mats)
    assert np.array_equal(k0, k1) and np.max(np.abs(a1 - a0)) < 1e-15
    for t in (2, 3):
        k2, _, a2 = _run_ops(c, [wl.make_op("ROT", 0, qmask=2, table=t, ctls=ctl)], mats)
        assert len(k2) == len(k0)
        assert np.allclose(np.sort(np.abs(a2)), np.sort(np.abs(a0)), rtol=0, atol=1e-15)
    kh, _, ah = _run_ops(c, [wl.make_op("H", 0, qmask=8, ctls=ctl)])
    kr, _, ar = _run_ops(c, [wl.make_op("ROT", 0, qmask=8, table=4, ctls=ctl)], mats)
    assert np.array_equal(kh, kr) and np.max(np.abs(ah - ar)) < 1e-16


@pytest.mark.parametrize("seed", range(3))
def test_arithmetic_oracle_inverses(seed):
    """ADDC(c) then ADDC(-c), MUL twice and DIV twice are the identity, bit for bit."""
    c = _start(seed, widths=(4, 3, 3, 2))
    k0, _, a0 = _run_ops(c, [])
    ops = [wl.make_op("ADDC", 0, imm=11, ctls=[(1, 2, 1)]), wl.make_op("ADDC", 0, imm=16 - 11, ctls=[(1, 2, 1)]),
           wl.make_op("MUL", 1, reg2=0, reg3=2), wl.make_op("MUL", 1, reg2=0, reg3=2),
           wl.make_op("DIV", 1, reg2=0, reg3=3, reg4=2), wl.make_op("DIV", 1, reg2=0, reg3=3, reg4=2)]
    k1, _, a1 = _run_ops(c, ops)
    assert np.array_equal(k0, k1) and np.array_equal(a0.view(np.uint64), a1.view(np.uint64))


def test_multiply_and_divide_closed_form():
    """On every basis state |x>|y>|0>|0> (x: 5 qubits, y: 3) MUL writes x*y
    mod 2^6 and DIV writes x div y and x mod y (all ones and x for y = 0)."""
    st = OracleState([("x", 5), ("y", 3), ("p", 6), ("q", 5), ("r", 3)])
    st.apply(wl.ops_array([wl.make_op("H", 0, qmask=0b11111), wl.make_op("H", 1, qmask=0b111),
                           wl.make_op("MUL", 2, reg2=0, reg3=1), wl.make_op("DIV", 3, reg2=0, reg3=1, reg4=4)]))
    _, v, a = st.export()
    assert len(v) == 256
    for x, y, p, q, r in v.tolist():
        assert p == (x * y) % 64
        assert (q, r) == ((x // y, x % y) if y else (31, x & 7))
    assert np.all(np.abs(a - 1 / 16) < 1e-16)


def _bitrev(y, n):
    return int(format(y, f"0{n}b")[::-1], 2)


@pytest.mark.parametrize("n,x", [(5, 0b10110), (8, 201), (11, 1234)])
def test_qft_closed_form(n, x):
    """Textbook QFT of |x> without the final swaps: amplitude of |y> is
    2^(-n/2) e^(2 pi i x rev(y) / 2^n) (rev: bit reversal); with the swaps,
    the same at y itself.  Pins the controlled phase gate and H together;
    also oracle against the dense checker."""
    for swaps in (False, True):
        c = wl.qft_circuit(n, x, swaps=swaps)
        st = _oracle_vs_dense(c, tol=1e-12)
        _, v, a = st.export()
        assert len(v) == 2 ** n
        ys = v[:, 0].astype(np.int64)
        yy = ys if swaps else np.array([_bitrev(int(y), n) for y in ys])
        expect = np.exp(2j * np.pi * ((x * yy) % 2 ** n) / 2 ** n) / 2 ** (n / 2)
        assert np.max(np.abs(a - expect)) < 1e-13
