"""Dynamic registers and the probability readout on the HIP path (through
the C ABI) against the oracle: registers added to a live state (in free bits,
in bits a removed register freed, and with keys gaining words, re-packed on
the device), removed when they hold one value, and probabilities of a
register without collapse, small, batched and at 2^21 entries."""
import numpy as np
import pytest

import workloads as wl
from oracle.closed_forms import c2_closed_form
from oracle.oracle import OracleState, run_circuit
from parity import compare, compare_arrays

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def abi():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2503_15118_amd import _abi
    return _abi


def _both(abi, regs, cap, init=None):
    st = abi.State(regs, cap_entries=cap, table_bytes=4096)
    ora = OracleState(regs, 1e-14)
    if init is not None:
        st.set_entries(0, *init)
        ora.set_entries(*init)
    return st, ora


def _apply(st, ora, ops):
    a = wl.ops_array(ops)
    st.apply(a)
    ora.apply(a)


def _same(st, ora):
    gk, ga = st.export()
    ok, _, oa = ora.export()
    return compare(gk, ga, ok, oa, 1e-14)


def test_add_registers_and_grow_key(abi):
    """a:60 in word 0; add 4 qubits (word 0), then 64 (a second word), then
    64 and 64 (four words): entries re-packed each time, ops on every
    register afterwards, against the oracle doing the same."""
    print("[case] add registers, keys 1 -> 2 -> 4 words", flush=True)
    st, ora = _both(abi, [("a", 60)], 1 << 18)
    _apply(st, ora, [wl.make_op("H", 0, qmask=(1 << 59) | 0b111111111 | (1 << 30)),
                     wl.make_op("MULC", 0, imm=0x5DEECE66D)])
    assert st.key_words == 1
    r1 = st.add_register(4)
    assert r1 == ora.add_register(4) == 1 and st.layout(1) == (0, 60, 4)
    _apply(st, ora, [wl.make_op("H", 1, qmask=0b11), wl.make_op("ADD", 1, reg2=0)])
    _same(st, ora)
    cap0 = st.capacity
    r2 = st.add_register(64)
    assert r2 == ora.add_register(64) and st.key_words == 2 and st.capacity < cap0
    _apply(st, ora, [wl.make_op("XOR", r2, reg2=0), wl.make_op("RY", r2, qmask=1 << 63, theta=0.8),
                     wl.make_op("X", 0, qmask=1, ctls=[(r2, 63, 1)])])
    _same(st, ora)
    r3 = st.add_register(64)
    r4 = st.add_register(64)
    assert (r3, r4) == (ora.add_register(64), ora.add_register(64)) and st.key_words == 4
    _apply(st, ora, [wl.make_op("ADD", r4, reg2=r2), wl.make_op("H", r3, qmask=1 << 40),
                     wl.make_op("MUL", r3, reg2=0, reg3=r4), wl.make_op("H", 1, qmask=0b1)])
    s = _same(st, ora)
    assert s["n_oracle"] > 4096
    with pytest.raises(RuntimeError):
        st.add_register(8)                         # 256 bits in use
    st.close()


def test_remove_register_and_reuse_bits(abi):
    print("[case] remove a register, reuse its bits", flush=True)
    st, ora = _both(abi, [("a", 6), ("tmp", 5), ("b", 6)], 1 << 12)
    _apply(st, ora, [wl.make_op("H", 0, qmask=0b111111), wl.make_op("XORC", 1, imm=21),
                     wl.make_op("ADD", 2, reg2=0)])
    with pytest.raises(RuntimeError):
        st.remove_register(0)                      # a varies
    st.remove_register(1)
    ora.remove_register(1)
    _same(st, ora)
    res = st.apply(abi.to_ss_ops(wl.ops_array([wl.make_op("X", 1, qmask=1)])), raise_on_error=False)
    assert res.status == abi.SS_E_ARG              # ops on a removed register
    r = st.add_register(5)
    assert r == ora.add_register(5) and st.layout(r)[:2] == (0, 6)
    _apply(st, ora, [wl.make_op("H", r, qmask=0b10001), wl.make_op("SUB", r, reg2=0)])
    _same(st, ora)
    st.close()


@pytest.mark.parametrize("seed", range(4))
def test_probabilities_small(abi, seed):
    c = wl.random_small_circuit(seed + 7, nops=60, with_init=bool(seed % 2))
    st = abi.state_for_circuit(c)
    st.apply(c.ops)
    k0, a0 = st.export()
    ora, _, _ = run_circuit(c)
    for reg in range(len(c.regs)):
        v, p = st.probabilities(0, reg)
        ov, op = ora.probabilities(reg)
        assert np.array_equal(v, ov) and np.max(np.abs(p - op)) <= 1e-12
    k1, a1 = st.export()
    assert np.array_equal(k0, k1) and np.array_equal(a0, a1)
    st.close()


def test_probabilities_batched_instance(abi):
    from paper_2503_15118_amd import batch
    circ = wl.c3_batch(9, ninst=5, lo_bits=8.0, hi_bits=12.0, len_lo=60, len_hi=100)
    st, _ = batch.run_batched(circ, cap_entries=1 << 20)
    for inst in (0, 3, 4):
        ora, _, _ = run_circuit(circ[inst])
        for reg in range(3):
            v, p = st.probabilities(inst, reg)
            ov, op = ora.probabilities(reg)
            assert np.array_equal(v, ov) and np.max(np.abs(p - op)) <= 1e-12
    st.close()


def test_probabilities_large(abi):
    """2^21 entries: the flag's two values and register b's ~2^20 values,
    against the closed form's marginals; nothing collapses."""
    import math
    c = wl.c2_circuit(6, nops=60, n_ry=2, h_qubits=20)
    print(f"[case] probabilities on {c.name}", flush=True)
    st = abi.state_for_circuit(c, cap_entries=1 << 22)
    st.apply(c.ops)
    ck, ca = c2_closed_form(c)
    mag = np.abs(ca) ** 2
    P = math.fsum(mag)
    for reg, word, shift, width in ((3, 1, 32, 1), (1, 0, 32, 32)):
        vals = (ck[:, word] >> np.uint64(shift)) & np.uint64((1 << width) - 1)
        uv, inv = np.unique(vals, return_inverse=True)
        if len(uv) <= 16:
            pv = np.array([math.fsum(mag[inv == j]) for j in range(len(uv))])
        else:
            pv = np.bincount(inv, weights=mag)
        v, p = st.probabilities(0, reg)
        assert np.array_equal(v, uv)
        n = len(ck)
        tol = max(1e-12, 2.0 * (n / 256 + 256) * 2.0 ** -53)
        assert np.max(np.abs(p - pv / P)) <= tol
    gk, ga = st.export()
    compare_arrays(gk, ga, ck, ca, c.eps)
    st.close()
