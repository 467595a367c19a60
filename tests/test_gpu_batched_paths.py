"""Batched rounds on the cases the round kernels treat apart: parents with
different child counts in one row of 64 (several instances per row, targets
on 1..5 qubits, controls that fail, so a parent has 1, 2 or up to 32
children; complex rotations), runs of equal keys up to 32 long in the
reduce, keys of two words, and a view of more than 2^20 entries (the run
launch's grid strides over it).  Every instance is compared with the oracle."""
import numpy as np
import pytest

import workloads as wl
from oracle.oracle import run_circuit
from parity import compare, compare_arrays

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def abi():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2503_15118_amd import _abi
    return _abi


# a general complex unitary (every element nonzero: the rotation branches)
_t, _p, _q = 0.7, 0.3, -1.1
ROTM = np.array([[np.cos(_t), -np.exp(1j * _p) * np.sin(_t)],
                 [np.exp(1j * _q) * np.sin(_t), np.exp(1j * (_p + _q)) * np.cos(_t)]], dtype=np.complex128)


def _mixed_circuits(regs, ninst, seed):
    """Instance i: H on (i % 5) + 1 qubits of a (controlled by a qubit of b for
    every third instance), a complex rotation on a qubit of b that an H made
    vary, a run (controlled X, ADD), then an H on the same qubits of a again
    (merges: runs of equal keys up to 32 long) and one more rotation."""
    rng = np.random.default_rng(seed)
    mk = wl.make_op
    wa = regs[0][1]
    out = []
    for i in range(ninst):
        k = i % 5 + 1
        qs = rng.choice(min(wa, 8), size=k, replace=False)
        qmask = 0
        for q in qs:
            qmask |= 1 << int(q)
        ctls = [(1, 2, 1)] if i % 3 == 0 else []
        ops = [mk("H", 1, qmask=1 << 2)]                      # b2 varies
        if i % 7 == 0:
            ops.append(mk("H", 1, qmask=0b11 << 4))           # a few more entries
        ops += [
            mk("H", 0, qmask=qmask, ctls=ctls),
            mk("ROT", 1, qmask=1 << 2, table=0),
            mk("X", 1, qmask=1 << 3, ctls=[(0, int(qs[0]), 1)]),
            mk("ADD", 1, reg2=0),
            mk("H", 0, qmask=qmask, ctls=ctls),               # merges back
            mk("ROT", 1, qmask=1 << 3, table=0),
        ]
        c = wl.Circuit(regs=regs, ops=wl.ops_array(ops), eps=1e-14, name=f"mixed-{i}")
        c.matrices = [ROTM]
        out.append(c)
    return out


@pytest.mark.parametrize("regs", [
    [("a", 8), ("b", 8), ("f", 1)],                       # one key word
    [("a", 30), ("b", 30), ("c", 20), ("f", 1)],          # two key words
], ids=["W1", "W2"])
def test_mixed_child_counts_match_oracle(abi, regs):
    from paper_2503_15118_amd import batch
    circ = _mixed_circuits(regs, 75, seed=5)
    print(f"[case] batched mixed child counts, {len(circ)} instances, regs {regs}", flush=True)
    st, res = batch.run_batched(circ, cap_entries=1 << 20)
    for i, c in enumerate(circ):
        gk, ga = st.export(i)
        ora, _, _ = run_circuit(c)
        ok, _, oa = ora.export()
        compare(gk, ga, ok, oa, c.eps)
    st.close()


def test_run_launch_strides_over_a_large_view(abi):
    """Instance 0 grows to 2^21 entries (H on 21 qubits of a, in chunks of
    five), then a run rewrites b from a; instance 1 stays one entry.  The
    final run covers 2^21 + 1 entries with a grid of 4096 workgroups."""
    from paper_2503_15118_amd import batch
    mk = wl.make_op
    regs = [("a", 21), ("b", 21)]
    big = wl.Circuit(regs=regs, ops=wl.ops_array([
        mk("H", 0, qmask=(1 << 21) - 1), mk("ADD", 1, reg2=0), mk("XORC", 1, imm=0x155),
        mk("X", 0, qmask=1 << 20, ctls=[(1, 0, 1)])]), eps=1e-14, name="big")
    small = wl.Circuit(regs=regs, ops=wl.ops_array([mk("X", 0, qmask=8), mk("ADD", 1, reg2=0)]),
                       eps=1e-14, name="small")
    circ = [big, small]
    print("[case] batched run over 2^21 + 1 entries", flush=True)
    st, res = batch.run_batched(circ, cap_entries=1 << 22)
    assert st.nnz() == (1 << 21) + 1
    for i, c in enumerate(circ):
        gk, ga = st.export(i)
        ora, _, _ = run_circuit(c)
        ok, _, oa = ora.export()
        compare_arrays(gk, ga, ok, oa, c.eps)
    st.close()
