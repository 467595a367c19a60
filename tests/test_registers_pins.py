"""Dynamic registers and the probability readout on the CPU oracle: adding a
register to a live state equals creating the state with it; removing a
register that holds one value equals a state without it; freed bits are
reused; keys gain a word when no word has room; probabilities match the
dense checker's marginals and leave the state unchanged."""
import numpy as np
import pytest

import workloads as wl
from oracle.dense import DenseState
from oracle.oracle import OracleState, run_circuit


def _vals(st):
    _, v, a = st.export()
    o = np.lexsort(v.T[::-1])
    return v[o], a[o]


def test_add_register_equals_created_with_it():
    c = wl.random_small_circuit(3, widths=(4, 3, 3), nops=40, with_init=True)
    grow = OracleState(c.regs, c.eps, c.tables, c.init_values, c.init_amps)
    grow.apply(c.ops[:20])
    r = grow.add_register(5)
    assert r == 3 and grow.layout(3) == (0, 10)
    full_init = np.concatenate([c.init_values, np.zeros((len(c.init_values), 1), dtype=np.uint64)], axis=1)
    full = OracleState(c.regs + [("new", 5)], c.eps, c.tables, full_init, c.init_amps)
    full.apply(c.ops[:20])
    more = wl.ops_array([wl.make_op("H", 3, qmask=0b101), wl.make_op("ADD", 3, reg2=0),
                         wl.make_op("X", 0, qmask=1, ctls=[(3, 2, 1)]), wl.make_op("RY", 3, qmask=2, theta=0.4)])
    ops2 = np.concatenate([c.ops[20:], more])
    grow.apply(ops2)
    full.apply(ops2)
    v1, a1 = _vals(grow)
    v2, a2 = _vals(full)
    assert np.array_equal(v1, v2) and np.array_equal(a1.view(np.uint64), a2.view(np.uint64))


def test_remove_register():
    st = OracleState([("a", 3), ("tmp", 4), ("b", 3)])
    st.apply(wl.ops_array([wl.make_op("H", 0, qmask=0b111), wl.make_op("XORC", 1, imm=9),
                           wl.make_op("ADD", 2, reg2=0)]))
    with pytest.raises(ValueError):
        st.remove_register(0)                     # a is in superposition
    st.remove_register(1)                         # tmp holds 9 everywhere
    v, a = _vals(st)
    ref = OracleState([("a", 3), ("b", 3)])
    ref.apply(wl.ops_array([wl.make_op("H", 0, qmask=0b111), wl.make_op("ADD", 1, reg2=0)]))
    rv, ra = _vals(ref)
    assert np.array_equal(v[:, [0, 2]], rv) and np.all(v[:, 1] == 0) and np.array_equal(a, ra)
    # the freed bits (3..6) take the next register of at most 4 qubits
    r = st.add_register(4)
    assert st.layout(r) == (0, 3)
    r2 = st.add_register(60)                      # no room in word 0: a second word
    assert st.layout(r2) == (1, 0)
    k, _, _ = st.export()
    assert np.all(k[:, 1] == 0)


def test_key_gains_words():
    st = OracleState([("a", 60)])
    st.apply(wl.ops_array([wl.make_op("H", 0, qmask=(1 << 59) | 1)]))
    ids = [st.add_register(w) for w in (64, 64, 64)]
    assert [st.layout(r) for r in ids] == [(1, 0), (2, 0), (3, 0)]
    st.apply(wl.ops_array([wl.make_op("XOR", 3, reg2=0), wl.make_op("H", 2, qmask=1 << 63)]))
    k, v, a = st.export()
    assert len(k) == 8 and set(v[:, 3].tolist()) == set(v[:, 0].tolist())
    with pytest.raises(ValueError):
        st.add_register(8)                        # four words full


@pytest.mark.parametrize("seed", range(5))
def test_probabilities_match_dense_marginals(seed):
    c = wl.random_small_circuit(seed, nops=50, with_init=bool(seed % 2))
    st, _, _ = run_circuit(c)
    k0, _, a0 = st.export()
    d = DenseState.from_circuit(c)
    d.apply(c.ops)
    for reg in range(len(c.regs)):
        v, p = st.probabilities(reg)
        idx = np.arange(len(d.v), dtype=np.uint64)
        f = d.field(idx, reg).astype(np.int64)
        marg = np.bincount(f, weights=np.abs(d.v) ** 2, minlength=2 ** c.regs[reg][1])
        marg = marg / marg.sum()
        nz = np.flatnonzero(marg > 0)
        assert np.array_equal(v.astype(np.int64), nz)
        assert np.max(np.abs(p - marg[nz])) < 1e-14
        assert abs(p.sum() - 1.0) < 1e-14
    k1, _, a1 = st.export()
    assert np.array_equal(k0, k1) and np.array_equal(a0.view(np.uint64), a1.view(np.uint64))
