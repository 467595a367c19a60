"""Batched rounds retire finished instances: the instances are relabelled so
that labels ascend with the pass of their last op, and after every round the
finished ones (a prefix of the sorted entries) leave the rounds.  Results are
bit-identical with retirement off; the labels and the full array come back at
the end of the call, after a capacity failure inside the rounds and after a
graph replay whose plan check fails inside them."""
import numpy as np
import pytest

import workloads as wl
from oracle.oracle import OracleState, run_circuit
from parity import compare

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def abi():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2503_15118_amd import _abi
    return _abi


def _exports(st, n):
    return [st.export(i) for i in range(n)]


def _bits_equal(x, y):
    (k1, a1), (k0, a0) = x, y
    assert np.array_equal(k1, k0)
    assert np.array_equal(a1.view(np.uint64), a0.view(np.uint64))


def test_retire_matches_no_retire_bit_for_bit(abi):
    from paper_2503_15118_amd import batch
    circ = wl.c3_batch(11, ninst=48, lo_bits=4.0, hi_bits=11.0, len_lo=30, len_hi=200)
    print(f"[case] retire on/off, {len(circ)} instances", flush=True)
    outs = []
    for r in (1, 0):
        st = batch.batch_state(circ, cap_entries=1 << 18)
        st.set_option("retire", r)
        ops, off = batch.concat_ops(circ)
        st.apply(ops, inst_offsets=off)
        outs.append(_exports(st, len(circ)))
        st.close()
    for x, y in zip(*outs):
        _bits_equal(x, y)
    for i in (0, 7, 23, 47):
        ora, _, _ = run_circuit(circ[i])
        ok, _, oa = ora.export()
        compare(outs[0][i][0], outs[0][i][1], ok, oa, circ[i].eps)


def _h_add_circuit(regs, nh):
    """nh rounds of (H on a fresh qubit of a, then b += a): one branching op
    per round, and a run after each one."""
    ops = []
    for q in range(nh):
        ops.append(wl.make_op("H", 0, qmask=1 << q))
        ops.append(wl.make_op("ADD", 1, reg2=0))
    return wl.Circuit(regs=regs, ops=wl.ops_array(ops), eps=1e-14)


def test_capacity_failure_restores_labels(abi):
    """Instance 0 doubles every round and overflows 256 entries in round 8,
    after instances 1..3 finished and were retired (rounds 2 and 3): the call
    fails with SS_E_CAPACITY naming the round, and every instance holds
    exactly what it had at that round's input (instance 0: its first 7 H and
    7 ADD; the others: their whole list), under its own instance id."""
    from paper_2503_15118_amd import batch
    regs = [("a", 12), ("b", 12)]
    circ = [_h_add_circuit(regs, n) for n in (10, 1, 2, 1)]
    st = batch.batch_state(circ, cap_entries=256)
    assert st.capacity < 264
    ops, off = batch.concat_ops(circ)
    print("[case] batched capacity failure after retirement", flush=True)
    res = st.apply(ops, inst_offsets=off, raise_on_error=False)
    assert res.status == abi.SS_E_CAPACITY and res.failed_op == 8, (res.status, res.failed_op)
    r = int(res.failed_op)
    for i, c in enumerate(circ):
        want = c.ops[:2 * (r - 1)] if i == 0 else c.ops
        ora = OracleState(regs, c.eps)
        ora.apply(want)
        ok, _, oa = ora.export()
        k, a = st.export(i)
        compare(k, a, ok, oa, c.eps)
    # the state is whole again: a plain op on instance 0 runs and the
    # retired instances are untouched by it
    before = _exports(st, len(circ))
    st.apply(abi.to_ss_ops(wl.ops_array([wl.make_op("X", 1, qmask=1)])), inst_offsets=np.array(
        [0, 1, 1, 1, 1], dtype=np.uint64))
    for i in (1, 2, 3):
        _bits_equal(st.export(i), before[i])
    st.close()


def test_failed_replay_restores_labels(abi):
    """Captured with every instance at |0>; replayed where instance 2 starts
    at b = 5, so the bits that vary after the first round differ from the
    recording and the plan check fails there.  The replay rolls back to the
    first round's input (no op has run: every list starts with H) and the
    labels come back: every instance holds exactly its starting entry."""
    from paper_2503_15118_amd import batch
    regs = [("a", 6), ("b", 6)]
    circ = [_h_add_circuit(regs, n) for n in (3, 1, 4, 2)]
    st = batch.batch_state(circ, cap_entries=1 << 12)
    ops, off = batch.concat_ops(circ)
    print("[case] failed batched replay", flush=True)
    g = st.capture(ops, inst_offsets=off)
    starts = []
    for i in range(len(circ)):
        v = np.zeros((1, 2), dtype=np.uint64)
        if i == 2:
            v[0, 1] = 5
        st.set_entries(i, v, np.array([1.0 + 0j]))
        starts.append(st.export(i))
    res = g.launch(raise_on_error=False)
    assert res.status == abi.SS_E_PLAN, res.status
    for i in range(len(circ)):
        _bits_equal(st.export(i), starts[i])
    # and the state runs the list eagerly from there
    st.apply(ops, inst_offsets=off)
    for i, c in enumerate(circ):
        ora = OracleState(regs, c.eps)
        v = np.zeros((1, 2), dtype=np.uint64)
        if i == 2:
            v[0, 1] = 5
        ora.set_entries(v, np.array([1.0 + 0j]))
        ora.apply(c.ops)
        ok, _, oa = ora.export()
        k, a = st.export(i)
        compare(k, a, ok, oa, c.eps)
    g.close()
    st.close()
