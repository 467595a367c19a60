"""Captured op lists (HIP graphs) through the C ABI.

A capture applies the ops (its result must equal eager application and the
oracle); every replay, with the program's own eager work and synchronisations
between replays, must equal that result bit for bit.  A replay on a state the
plan does not fit must return SS_E_PLAN with the state rolled back to an op
boundary, from where eager application finishes the job.
"""
import numpy as np
import pytest

import workloads as wl
from oracle.oracle import OracleState, run_circuit
from parity import compare

pytestmark = pytest.mark.gpu

H = 0.70710678118654752440


@pytest.fixture(scope="module")
def abi():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2503_15118_amd import _abi
    return _abi


def _init(c):
    v = c.init_values if c.init_values is not None else np.zeros((1, len(c.regs)), dtype=np.uint64)
    a = c.init_amps if c.init_amps is not None else np.array([1.0 + 0j])
    return v, a


def _same(x, y):
    (k1, a1), (k0, a0) = x, y
    assert np.array_equal(k1, k0)
    assert np.array_equal(a1.view(np.uint64), a0.view(np.uint64))


def _circuit(form, seed):
    if form == "c1":
        return wl.c1_circuit(seed)
    if form == "c2":
        # H on 12 qubits: split over three launches, checks between them
        return wl.c2_circuit(seed, nops=200, n_ry=4, h_qubits=12)
    return wl.random_small_circuit(seed, nops=80, with_init=True)


@pytest.mark.parametrize("form,seed", [("c1", 0), ("c1", 1), ("c2", 2), ("small", 3), ("small", 4)])
def test_replays_equal_eager_and_oracle(abi, form, seed):
    c = _circuit(form, seed)
    print(f"[case] graph {c.name} nops={len(c.ops)}", flush=True)
    ops = abi.to_ss_ops(c.ops)
    v, a = _init(c)
    st = abi.state_for_circuit(c)
    g = st.capture(ops)
    first = st.export()
    ora, _, _ = run_circuit(c)
    ok, _, oa = ora.export()
    compare(first[0], first[1], ok, oa, c.eps)
    ref = abi.state_for_circuit(c)
    ref.apply(ops)
    _same(first, ref.export())
    ref.close()
    for rep in range(3):
        st.set_entries(0, v, a)
        res = g.launch()
        assert res.status == 0
        _same(st.export(), first)
        assert st.nnz() == len(first[0])
    # eager application after replays (ring and look-back tags handed back)
    st.set_entries(0, v, a)
    st.apply(ops)
    _same(st.export(), first)
    # and a replay after eager work again
    st.set_entries(0, v, a)
    g.launch()
    _same(st.export(), first)
    g.close()
    st.close()


def test_batched_replays(abi):
    from paper_2503_15118_amd import batch
    circ = wl.c3_batch(5, ninst=8, lo_bits=4.0, hi_bits=10.0, len_lo=40, len_hi=120)
    print(f"[case] graph batched {len(circ)} instances", flush=True)
    st = batch.batch_state(circ, cap_entries=1 << 17)
    ops, off = batch.concat_ops(circ)
    g = st.capture(ops, inst_offsets=off)
    first = [st.export(i) for i in range(len(circ))]
    for i, c in enumerate(circ):
        ora, _, _ = run_circuit(c)
        ok, _, oa = ora.export()
        compare(first[i][0], first[i][1], ok, oa, c.eps)
    for rep in range(2):
        for i, c in enumerate(circ):
            v, a = _init(c)
            st.set_entries(i, v, a)
        g.launch()
        for i in range(len(circ)):
            _same(st.export(i), first[i])
    g.close()
    st.close()


def test_count_mismatch_refused_before_launch(abi):
    c = wl.random_small_circuit(7, nops=60, with_init=True)
    ops = abi.to_ss_ops(c.ops)
    st = abi.state_for_circuit(c)
    g = st.capture(ops)
    v, a = _init(c)
    assert len(v) >= 2
    # one entry fewer: refused, nothing runs
    st.set_entries(0, v[:-1], a[:-1] / np.linalg.norm(a[:-1]))
    before = st.export()
    res = g.launch(raise_on_error=False)
    assert res.status == abi.SS_E_PLAN and res.failed_op == 0
    _same(st.export(), before)
    g.close()
    st.close()


def test_mask_mismatch_rolls_back_and_resumes(abi):
    """Captured on {a=0, a=4} (bit 2 varies; H on bit 1 is a pure expansion),
    replayed on {a=0, a=2} (bit 1 varies): the check before H fails, the state
    holds the result of the X, and eager application of the rest matches the
    oracle."""
    regs = [("a", 3)]
    ops_n = wl.ops_array([wl.make_op("X", 0, qmask=1), wl.make_op("H", 0, qmask=2),
                          wl.make_op("X", 0, qmask=4)])
    ops = abi.to_ss_ops(ops_n)
    amps = np.array([H + 0j, H + 0j])
    st = abi.State(regs, cap_entries=1 << 10, table_bytes=0)
    st.set_entries(0, np.array([[0], [4]], dtype=np.uint64), amps)
    g = st.capture(ops)
    vals = np.array([[0], [2]], dtype=np.uint64)
    st.set_entries(0, vals, amps)
    res = g.launch(raise_on_error=False)
    assert res.status == abi.SS_E_PLAN
    assert res.failed_op == 1
    k, a = st.export()
    assert sorted(int(x) for x in k[:, 0]) == [1, 3]
    st.apply(ops[1:])
    gk, ga = st.export()
    o = OracleState(regs, 1e-14, init_values=vals, init_amps=amps)
    o.apply(ops_n)
    ok, _, oa = o.export()
    compare(gk, ga, ok, oa, 1e-14)
    # the graph still works on a state that fits
    st.set_entries(0, np.array([[0], [4]], dtype=np.uint64), amps)
    assert g.launch().status == 0
    g.close()
    st.close()


def test_graph_outliving_state_is_refused(abi):
    c = wl.c1_circuit(3)
    st = abi.state_for_circuit(c)
    g = st.capture(abi.to_ss_ops(c.ops))
    st.close()
    res = g.launch(raise_on_error=False)
    assert res.status == abi.SS_E_STATE
    g.close()


def test_capture_empty_state_and_rebind_refused(abi):
    """An empty state captures a graph that does nothing and replays cleanly;
    a graph of a state that moved to another arena is refused."""
    c = wl.random_small_circuit(9, nops=40, with_init=True)
    ops = abi.to_ss_ops(c.ops)
    st = abi.state_for_circuit(c)
    st.set_entries(0, np.zeros((0, len(c.regs)), dtype=np.uint64), np.zeros(0, dtype=np.complex128))
    g = st.capture(ops)
    assert st.nnz() == 0
    assert g.launch().status == 0 and st.nnz() == 0
    g.close()
    v, a = _init(c)
    st.set_entries(0, v, a)
    g = st.capture(ops)
    want = st.export()
    st.rebind(st.capacity * 2)
    res = g.launch(raise_on_error=False)
    assert res.status == abi.SS_E_ARG
    _same(st.export(), want)              # the refused launch changed nothing
    g.close()
    st.close()
