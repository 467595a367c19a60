"""HIP path vs the CPU oracle, element by element, through the C ABI.

Keys outside the band |a| <= eps + 1e-9 must match word for word; shared keys
within 1e-12 (complex modulus); export must be strictly ascending.
"""
import numpy as np
import pytest

import workloads as wl
from oracle.oracle import OracleState, run_circuit
from parity import compare

pytestmark = pytest.mark.gpu

C = 0.70710678118654752440


@pytest.fixture(scope="module")
def abi():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2503_15118_amd import _abi
    return _abi


def _gpu(abi, c, cap=None, opts=None, ops=None):
    st = abi.state_for_circuit(c, cap_entries=cap)
    for k, v in (opts or {}).items():
        st.set_option(k, v)
    st.apply(c.ops if ops is None else ops)
    return st


def _check(abi, c, cap=None, opts=None, atol=1e-12):
    print(f"[case] {c.name} nops={len(c.ops)} opts={opts}", flush=True)
    st = _gpu(abi, c, cap, opts)
    gk, ga = st.export()
    ora, _, _ = run_circuit(c)
    ok, _, oa = ora.export()
    s = compare(gk, ga, ok, oa, c.eps, atol=atol)
    assert st.nnz() == len(gk)
    st.close()
    return s


def test_permutation_only_bit_exact(abi):
    """Minimum slice: non-branching ops on an imported superposition are
    bit-exact in keys and amplitudes."""
    kinds = ("X", "ADD", "SUB", "MULC", "XOR", "XORC", "QRAM_LOAD", "QRAM_UNLOAD", "REFLECT0")
    for seed in range(4):
        c = wl.random_small_circuit(seed, kinds=kinds, nops=80, with_init=True)
        s = _check(abi, c)
        assert s["bit_exact"] == s["shared"] == s["n_oracle"]


@pytest.mark.parametrize("seed", range(12))
def test_small_circuits_all_kinds(abi, seed):
    c = wl.random_small_circuit(seed, with_init=bool(seed % 2), eps=(0.0 if seed % 4 == 3 else 1e-14))
    _check(abi, c)


@pytest.mark.parametrize("seed", range(32))
def test_c1_form(abi, seed):
    c = wl.c1_circuit(seed)
    s = _check(abi, c)
    assert s["n_oracle"] > 1


@pytest.mark.parametrize("seed", range(3))
def test_c1_form_always_sort(abi, seed):
    """The plain method (sort before every interference op) gives the same state."""
    c = wl.c1_circuit(100 + seed)
    _check(abi, c, opts={"grouping": 0})
    _check(abi, c, opts={"grouping": 0, "sort_items": 8})


@pytest.mark.parametrize("nq", [23, 40, 255])
def test_ghz_two_branches(abi, nq):
    c = wl.ghz_circuit(nq)
    st = _gpu(abi, c)
    k, a = st.export()
    assert len(k) == 2
    assert np.all(a == C)
    _check(abi, c)


@pytest.mark.parametrize("ab,wb", [(4, 6), (10, 10), (12, 32)])
def test_qram_closed_form(abi, ab, wb):
    c = wl.qram_circuit(ab, ab, wb)
    _check(abi, c)
    st = _gpu(abi, c)
    k, a = st.export()
    assert len(k) == 2 ** ab
    expect = 1.0
    for _ in range(ab):
        expect = C * expect
    assert np.all(a == expect)


def test_c2_form_small(abi):
    c = wl.c2_circuit(3, nops=300, n_ry=5, h_qubits=10)
    _check(abi, c)
    _check(abi, c, opts={"grouping": 0})


def test_c4_form_batched_instances(abi):
    circ = wl.c4_batch(2, nrhs=4, steps=4, n=64)
    c0 = circ[0]
    st = abi.State(c0.regs, ninst=len(circ), eps=c0.eps, cap_entries=1 << 14, table_bytes=1 << 16)
    st.load_qram(c0.tables[0])
    for i, c in enumerate(circ):
        st.set_entries(i, c.init_values, c.init_amps)
    st.apply(c0.ops)
    for i, c in enumerate(circ):
        gk, ga = st.export(i)
        ora, _, _ = run_circuit(c)
        ok, _, oa = ora.export()
        compare(gk, ga, ok, oa, c.eps)
    st.close()


@pytest.mark.parametrize("seed", range(4))
def test_measure_matches_oracle(abi, seed):
    c = wl.random_small_circuit(seed, nops=30, with_init=True)
    reg = seed % len(c.regs)
    u = [0.13, 0.37, 0.61, 0.89][seed]
    st = _gpu(abi, c)
    ora, _, _ = run_circuit(c)
    v_g, p_g = st.measure(0, reg, u)
    v_o, p_o = ora.measure(reg, u)
    assert v_g == v_o
    assert abs(p_g - p_o) < 1e-12
    gk, ga = st.export()
    ok, _, oa = ora.export()
    compare(gk, ga, ok, oa, c.eps)


def test_prune_matches_oracle(abi):
    c = wl.random_small_circuit(5, nops=40, with_init=True, eps=0.0)
    st = _gpu(abi, c)
    ora, _, _ = run_circuit(c)
    for eps in (1e-3, 1e-2, 0.05):
        st.prune(eps)
        ora.prune(eps)
        gk, ga = st.export()
        ok, _, oa = ora.export()
        compare(gk, ga, ok, oa, eps)


def test_empty_state_and_noop(abi):
    c = wl.random_small_circuit(7, nops=20, with_init=True)
    st = _gpu(abi, c)
    st.prune(10.0)
    assert st.nnz() == 0
    st.apply(c.ops)
    assert st.nnz() == 0
    k, a = st.export()
    assert len(k) == 0


def test_capacity_error_rolls_back(abi):
    """An op whose survivors exceed the capacity fails with SS_E_CAPACITY and
    leaves the state as it was after the ops before it."""
    c = wl.c2_circuit(1, nops=10, n_ry=1, h_qubits=12)
    st = abi.State(c.regs, eps=c.eps, cap_entries=4096, table_bytes=0)
    assert 4096 <= st.capacity < 8192
    res = st.apply(c.ops, raise_on_error=False)
    assert res.status == abi.SS_E_CAPACITY
    assert wl.KINDS[int(c.ops[res.failed_op]["kind"])] == "RY"
    gk, ga = st.export()
    ora, _, _ = run_circuit(c, ops=c.ops[:res.failed_op])
    ok, _, oa = ora.export()
    s = compare(gk, ga, ok, oa, c.eps)
    assert s["n_gpu"] == 4096
    # an op split over several launches is refused before it starts
    st2 = abi.State(c.regs, eps=c.eps, cap_entries=4096, table_bytes=0)
    res = st2.apply(wl.ops_array([wl.make_op("H", 0, qmask=(1 << 14) - 1)]), raise_on_error=False)
    assert res.status == abi.SS_E_CAPACITY and res.failed_op == 0
    k, a = st2.export()
    assert len(k) == 1 and a[0] == 1.0


def test_capacity_failure_mid_stream_then_resume(abi):
    """A capacity failure inside a run of launches that the host queued
    without waiting: the launches after it change nothing, the state returns
    to the failing op's input, and after moving to a larger arena the rest of
    the ops give the oracle's result for the whole list."""
    regs = [("a", 8), ("b", 8)]
    ops = wl.ops_array([
        wl.make_op("H", 0, qmask=0xFF),                  # 256 entries (two launches)
        wl.make_op("ADD", 1, reg2=0),                    # b = a
        wl.make_op("RY", 1, qmask=0x0F, theta=0.7),      # 16 children each: 4096 > capacity
        wl.make_op("X", 0, qmask=1),
        wl.make_op("RY", 1, qmask=0x0F, theta=-0.7),     # same targets: no wait before it
        wl.make_op("XORC", 1, imm=0x35),
        wl.make_op("H", 0, qmask=0x03),
    ])
    c = wl.Circuit(name="cap-mid", regs=regs, ops=ops, eps=1e-14)
    print("[case] capacity mid-stream", flush=True)
    st = abi.State(regs, eps=c.eps, cap_entries=1024, table_bytes=0)
    cap = st.capacity
    assert 1024 <= cap < 4096
    res = st.apply(ops, raise_on_error=False)
    assert res.status == abi.SS_E_CAPACITY and res.failed_op == 2
    gk, ga = st.export()
    ora, _, _ = run_circuit(c, ops=ops[:2])
    ok, _, oa = ora.export()
    s = compare(gk, ga, ok, oa, c.eps)
    assert s["n_gpu"] == 256 and res.nnz == 256
    assert st.peak() == 256
    st.rebind(1 << 14)
    res = st.apply(ops[2:], raise_on_error=False)
    assert res.status == 0, abi.strerror(res.status)
    gk, ga = st.export()
    ora, _, _ = run_circuit(c)
    ok, _, oa = ora.export()
    compare(gk, ga, ok, oa, c.eps)
    st.close()


@pytest.mark.parametrize("seed", range(3))
def test_speculative_placement_is_exact(abi, seed):
    """One-target interference ops first try the fixed-fan-out placement; on
    circuits with controls (some entries pass through, some pairs are
    incomplete) and on the arithmetic-heavy form (full pairs) the result must
    equal, bit for bit and in the same order, the compacting path alone."""
    for c in (wl.c1_circuit(seed), wl.c2_circuit(seed, nops=60, n_ry=6, h_qubits=10),
              wl.random_small_circuit(seed, nops=80, with_init=True)):
        print(f"[case] {c.name} speculation on/off", flush=True)
        outs = []
        # 1: speculate at any size (expansions; grouped entries too, with each
        # way of finding partners and tile size)
        for opts in ({"speculate": 1, "speculate_group": 1, "pair_exchange": 2, "spec_items": 8},
                     {"speculate": 1, "speculate_group": 1, "pair_exchange": 2, "spec_items": 4},
                     {"speculate": 1, "speculate_group": 1, "pair_exchange": 1, "spec_items": 2},
                     {"speculate": 1, "speculate_group": 1, "pair_exchange": 0, "spec_items": 1},
                     {"speculate": 1, "speculate_group": 0}, {"speculate": 0, "speculate_group": 0}):
            st = _gpu(abi, c, opts=opts)
            outs.append(st.export())
            st.close()
        k0, a0 = outs[-1]
        for k1, a1 in outs[:-1]:
            assert np.array_equal(k1, k0)
            assert np.array_equal(a1.view(np.uint64), a0.view(np.uint64))
        k1, a1 = outs[0]
        ora, _, _ = run_circuit(c)
        ok, _, oa = ora.export()
        compare(k1, a1, ok, oa, c.eps)


@pytest.mark.parametrize("form", ["pure", "controlled", "varying"])
def test_many_target_expansions(abi, form):
    """H / Ry on 6..10 target qubits of one register: as one launch of one
    thread per child when no target bit can vary (with and without a control
    that fails for some entries), in launches of at most 5 targets with
    grouping when some do; all against the oracle, and the one-launch path
    against the one-thread-per-entry path of at most 5 targets."""
    mk = wl.make_op
    regs = [("a", 10), ("b", 4), ("f", 1)]
    rng = np.random.default_rng(90 + len(form))
    ops = [mk("H", 1, qmask=0xF)]
    if form == "varying":
        ops.append(mk("H", 0, qmask=0b1000100))            # targets 2 and 6 now vary
    ctls = [(1, 2, 1)] if form == "controlled" else []
    ops.append(mk("H", 0, qmask=0x3FF, ctls=ctls))
    ops.append(mk("ADD", 0, reg2=1))
    ops.append(mk("RY", 0, qmask=0x3F0, theta=float(rng.uniform(0, 6.28))))
    c = wl.Circuit(regs=regs, ops=wl.ops_array(ops), eps=1e-14, name=f"many-targets-{form}")
    # (an op split over several launches is admitted when n 2^k fits)
    s = _check(abi, c, cap=1 << 21)
    assert s["n_oracle"] > 0
    outs = []
    for opts in ({}, {"expand_slots": 0}):
        st = _gpu(abi, c, cap=1 << 21, opts=opts)
        outs.append(st.export())
        st.close()
    (k1, a1), (k0, a0) = outs
    compare(k1, a1, k0, a0, c.eps)


def test_wasted_speculation_cools_down(abi):
    """H on a flag qubit again and again: every expansion fits the fixed
    placement and every merge defeats it.  After a wasted speculative launch
    the next ones skip themselves, so only a few are wasted over 400 eligible
    ops; the result equals the compacting path bit for bit."""
    mk = wl.make_op
    regs = [("a", 6), ("f", 1)]
    ops = [mk("H", 0, qmask=0x3F)]
    for i in range(200):
        ops += [mk("H", 1, qmask=1), mk("X", 0, qmask=1 << (i % 6))]
    c = wl.Circuit(regs=regs, ops=wl.ops_array(ops), eps=1e-14, name="flag-h-pairs")
    print(f"[case] {c.name} wasted speculation", flush=True)
    outs = []
    for opts in ({"speculate": 1, "speculate_group": 1}, {"speculate": 0, "speculate_group": 0}):
        st = _gpu(abi, c, opts=opts)
        outs.append(st.export() + (st.stats()["speculation_wasted"],))
        st.close()
    (k1, a1, w1), (k0, a0, w0) = outs
    assert np.array_equal(k1, k0)
    assert np.array_equal(a1.view(np.uint64), a0.view(np.uint64))
    assert w0 == 0 and 1 <= w1 <= 20, w1
    ora, _, _ = run_circuit(c)
    ok, _, oa = ora.export()
    compare(k1, a1, ok, oa, c.eps)


def test_deterministic_reruns(abi):
    c = wl.c1_circuit(9)
    k1, a1 = _gpu(abi, c).export()
    k2, a2 = _gpu(abi, c).export()
    assert np.array_equal(k1, k2)
    assert np.array_equal(a1.view(np.uint64), a2.view(np.uint64))


def test_invalid_ops_rejected(abi):
    st = abi.State([("a", 4), ("b", 4)], cap_entries=1024)
    bad = [
        wl.make_op("X", 0, qmask=1 << 5),                      # qubit outside the register
        wl.make_op("ADD", 0, reg2=0),                          # dst == src
        wl.make_op("MULC", 0, imm=4),                          # even multiplier
        wl.make_op("X", 0, qmask=1, ctls=[(0, 0, 1)]),         # control on the target
        wl.make_op("ADD", 0, reg2=1, ctls=[(0, 2, 1)]),        # control inside dst
    ]
    codes = [abi.SS_E_ARG, abi.SS_E_ARG, abi.SS_E_NOT_UNITARY, abi.SS_E_ARG, abi.SS_E_ARG]
    for op, code in zip(bad, codes):
        res = st.apply(wl.ops_array([op]), raise_on_error=False)
        assert res.status == code
    assert st.nnz() == 1


def _c2_sample_check(abi, c, st, nsamp=48, seed=0):
    """Sampled parity at full size: the oracle evolves single trajectories
    (each C2-form branch only ever meets its flag partner)."""
    gk, ga = st.export()
    hop = c.ops[:1]
    ora0 = OracleState(c.regs, c.eps)
    ora0.apply(hop)
    _, v0, a0 = ora0.export()
    rng = np.random.default_rng(seed)
    idx = rng.choice(len(v0), size=nsamp, replace=False)
    w1 = gk[:, 1]
    checked = 0
    for i in idx:
        o = OracleState(c.regs, c.eps, init_values=v0[i:i + 1], init_amps=a0[i:i + 1])
        o.apply(c.ops[1:])
        ok, _, oa = o.export()
        for key, amp in zip(ok, oa):
            lo = np.searchsorted(w1, key[1], side="left")
            hi = np.searchsorted(w1, key[1], side="right")
            j = lo + np.searchsorted(gk[lo:hi, 0], key[0])
            assert j < hi and gk[j, 0] == key[0] and gk[j, 1] == key[1], "sampled key missing on GPU"
            assert abs(ga[j] - amp) <= 1e-12
            checked += 1
    return checked


@pytest.mark.slow
def test_c2_full_size_sampled(abi):
    """C2 at its full size (2^20 -> 2^21 entries, 1000 ops) in the benchmark's
    launch configuration: nnz exact, norm 1, sampled trajectories vs oracle."""
    c = wl.c2_circuit(0)
    print(f"[case] {c.name} full size", flush=True)
    st = abi.state_for_circuit(c, cap_entries=1 << 22)
    st.apply(c.ops)
    assert st.nnz() == 2 ** 21
    gk, ga = st.export()
    norm = float(np.sum(ga.real ** 2 + ga.imag ** 2))
    assert abs(norm - 1.0) < 1e-10
    assert _c2_sample_check(abi, c, st) >= 48


def test_reversed_pairs_after_flip(abi):
    """Grouped order survives an X on the target qubit with each pair reversed
    (bit 1 before bit 0); the next interference op on that qubit must find the
    partner on either side."""
    for ctl in ([], [(1, 0, 1)]):
        ops = wl.ops_array([
            wl.make_op("H", 1, qmask=0b111),
            wl.make_op("RY", 0, qmask=1 << 2, theta=0.9),
            wl.make_op("X", 0, qmask=1 << 2, ctls=ctl),
            wl.make_op("RY", 0, qmask=1 << 2, theta=2.1),
            wl.make_op("X", 0, qmask=(1 << 2) | 1),
            wl.make_op("H", 0, qmask=1 << 2),
        ])
        c = wl.Circuit(regs=[("a", 4), ("b", 3)], ops=ops, name=f"reversed-pairs-ctl{len(ctl)}")
        _check(abi, c)


@pytest.mark.parametrize("seed", [0, 1])
def test_batched_instances_match_oracle_and_plain(abi, seed):
    """Per-instance op lists in one state: each instance equals the oracle and
    its own plain single-instance run."""
    from paper_2503_15118_amd import batch
    circ = wl.c3_batch(seed, ninst=12, lo_bits=4.0, hi_bits=11.0, len_lo=40, len_hi=160)
    print(f"[case] batched c3-form seed {seed}: {len(circ)} instances", flush=True)
    st, res = batch.run_batched(circ, cap_entries=1 << 18)
    plain = batch.run_sequential(circ, cap_entries=1 << 14)
    for i, c in enumerate(circ):
        gk, ga = st.export(i)
        ora, _, _ = run_circuit(c)
        ok, _, oa = ora.export()
        compare(gk, ga, ok, oa, c.eps)
        pk, pa = plain[i]
        compare(gk, ga, pk, pa, c.eps)


def test_batched_mixed_kinds(abi):
    """Batched rounds with every op kind (random small circuits, QRAM table
    shared), uneven lengths including an empty op list."""
    from paper_2503_15118_amd import batch
    base = wl.random_small_circuit(3, nops=1)
    circ = []
    for i in range(6):
        c = wl.random_small_circuit(100 + i, nops=[30, 0, 55, 12, 41, 25][i], max_h=5)
        c.tables = base.tables
        circ.append(c)
    st, res = batch.run_batched(circ, cap_entries=1 << 16)
    for i, c in enumerate(circ):
        gk, ga = st.export(i)
        ora, _, _ = run_circuit(c)
        ok, _, oa = ora.export()
        compare(gk, ga, ok, oa, c.eps)


def test_host_superset_decisions(abi):
    """Expansions decided from the host's superset of varying key bits (no
    read-back): constant flips, controlled flips, arithmetic and imported
    superpositions must lead to the same state as the oracle."""
    mk = wl.make_op
    ops = wl.ops_array([
        mk("X", 0, qmask=1),                       # flip: q0 constant 1
        mk("H", 0, qmask=2),                       # q1 constant -> expansion
        mk("XORC", 0, imm=4),                      # flip q2
        mk("H", 0, qmask=4),                       # still constant -> expansion
        mk("X", 0, qmask=8, ctls=[(0, 1, 1)]),     # q3 varies now
        mk("H", 0, qmask=8),                       # needs the exact masks (grouped)
        mk("ADD", 1, reg2=0),                      # b += a: b varies
        mk("H", 1, qmask=1),
        mk("X", 1, qmask=2, ctls=[(0, 0, 0)]),     # control never true: q1 of b stays 0
        mk("H", 1, qmask=2),                       # superset says varying, exact says constant
        mk("H", 0, qmask=2),                       # q1 of a varies: group
        mk("RY", 2, qmask=1, theta=0.7),
    ])
    c = wl.Circuit(regs=[("a", 4), ("b", 3), ("f", 1)], ops=ops, name="superset")
    _check(abi, c)
    # imported superposition: the import's own masks say which bits vary
    vals = np.array([[0, 0, 0], [2, 0, 0], [2, 5, 0]], dtype=np.uint64)
    amps = np.array([0.6, 0.0 + 0.64j, 0.48], dtype=np.complex128)
    c2 = wl.Circuit(regs=[("a", 4), ("b", 3), ("f", 1)], ops=wl.ops_array([
        mk("H", 0, qmask=2), mk("H", 0, qmask=1), mk("H", 1, qmask=4), mk("H", 1, qmask=1),
        mk("RY", 2, qmask=1, theta=1.1)]), init_values=vals, init_amps=amps, name="superset-import")
    _check(abi, c2)


@pytest.mark.parametrize("entries", [4, 16])
def test_perm_entries_variants(abi, entries):
    """Entries per lane of the interpreter change the tiling only: every op
    kind on 1- and 2-word keys, with and without a phase op in the run."""
    kinds = ("X", "ADD", "SUB", "MULC", "XOR", "XORC", "QRAM_LOAD", "QRAM_UNLOAD", "REFLECT0")
    for seed in range(3):
        c = wl.random_small_circuit(40 + seed, kinds=kinds, nops=120, with_init=True)
        s = _check(abi, c, opts={"perm_entries": entries})
        assert s["bit_exact"] == s["shared"] == s["n_oracle"]
    _check(abi, wl.c2_circuit(6, nops=150, n_ry=3, h_qubits=12), opts={"perm_entries": entries})


def test_swap_test_form(abi):
    """Swap-test form: small size against the oracle; at the printed 25 qubits
    the peak equals the paper's branch count and the final state is the closed
    form (every (x, y) with the ancilla 0 and amplitude c^24)."""
    import json
    import os
    _check(abi, wl.swap_test_circuit(4))
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_branch_counts.json")))
    nq, branches = g["swap_test"][0]
    c = wl.swap_test_circuit((nq - 1) // 2)
    print(f"[case] {c.name} full size", flush=True)
    st = abi.state_for_circuit(c, cap_entries=1 << 26)
    st.apply(c.ops)
    assert st.peak() == branches
    k, a = st.export()
    assert len(k) == branches // 2
    assert np.array_equal(k[:, 0], np.arange(branches // 2, dtype=np.uint64))
    assert np.max(np.abs(a - C ** (nq - 1))) <= 1e-12
    st.close()


@pytest.mark.parametrize("seed", range(4))
def test_chained_one_target_ops(abi, seed):
    """Runs of H / Ry on one target qubit with varied controls (including
    none, H.H pairs and singleton groups) run as one launch: the result must
    match the oracle (which prunes after every op) and the unchained path."""
    rng = np.random.default_rng(500 + seed)
    mk = wl.make_op
    regs = [("a", 4), ("b", 3), ("f", 1)]
    ops = [mk("H", 0, qmask=0b0101)]
    for blk in range(6):
        reg, q = [(2, 0), (0, int(rng.integers(0, 4))), (1, int(rng.integers(0, 3)))][blk % 3]
        for _ in range(int(rng.integers(2, 20))):
            ctls = []
            for _c in range(int(rng.integers(0, 3))):
                cr = int(rng.integers(0, 3))
                cq = int(rng.integers(0, [4, 3, 1][cr]))
                if (cr, cq) != (reg, q) and all((cr, cq) != (x, y) for x, y, _ in ctls):
                    ctls.append((cr, cq, int(rng.integers(0, 2))))
            if rng.random() < 0.3:
                ops.append(mk("H", reg, qmask=1 << q, ctls=ctls))
            else:
                ops.append(mk("RY", reg, qmask=1 << q, theta=float(rng.uniform(0, 2 * np.pi)), ctls=ctls))
        ops.append(mk("ADD", 1, reg2=0))
        ops.append(mk("X", 0, qmask=1 << int(rng.integers(0, 4)), ctls=[(2, 0, 1)]))
    c = wl.Circuit(regs=regs, ops=wl.ops_array(ops), eps=(1e-14 if seed % 2 else 0.0), name=f"chains-{seed}")
    s1 = _check(abi, c, opts={"chain": 1})
    s0 = _check(abi, c, opts={"chain": 0})
    assert s1["n_oracle"] == s0["n_oracle"]
    st1 = _gpu(abi, c, opts={"chain": 1, "speculate": 0, "speculate_group": 0})
    st0 = _gpu(abi, c, opts={"chain": 0})
    k1, a1 = st1.export()
    k0, a0 = st0.export()
    compare(k1, a1, k0, a0, c.eps)
    # chains placed speculatively first (at any size): bit for bit the same
    st2 = _gpu(abi, c, opts={"chain": 1, "speculate": 1, "speculate_group": 1})
    k2, a2 = st2.export()
    assert np.array_equal(k2, k1)
    assert np.array_equal(a2.view(np.uint64), a1.view(np.uint64))
    st2.close()
    st1.close()
    st0.close()


@pytest.mark.parametrize("chunk", [7, 16])
def test_op_list_split_over_calls(abi, chunk):
    """The same circuit applied as many short calls: every call ends with a
    read-back and starts from the previous call's host view (grouping, masks,
    op-record ring), so chains, runs and their uploaded records meet
    synchronisations at every position.  Must equal the oracle."""
    for seed in (0, 3, 11):
        c = wl.c1_circuit(seed)
        print(f"[case] {c.name} in calls of {chunk} ops", flush=True)
        st = abi.state_for_circuit(c)
        ops = abi.to_ss_ops(c.ops)
        for a in range(0, len(ops), chunk):
            st.apply(ops[a:a + chunk])
        gk, ga = st.export()
        ora, _, _ = run_circuit(c)
        ok, _, oa = ora.export()
        compare(gk, ga, ok, oa, c.eps)
        st.close()


@pytest.mark.parametrize("items", [1, 2, 4])
def test_fused_runs_bit_identical(abi, items):
    """A one-target op that takes the following run of non-branching ops into
    its launch writes the same entries at the same positions as the two
    launches: keys and amplitudes bit for bit, and equal to the oracle.  Runs
    with every op kind (QRAM, phase) on 1- and 2-word keys, expansions and
    groups, chains and singletons; with the fixed-fan-out placement tried
    first (it carries the run too) and without."""
    kinds = ("X", "H", "RY", "ADD", "SUB", "MULC", "XOR", "XORC", "QRAM_LOAD", "QRAM_UNLOAD", "REFLECT0")
    circs = [wl.random_small_circuit(70 + s, kinds=kinds, nops=120, with_init=bool(s % 2)) for s in range(3)]
    circs += [wl.c1_circuit(21), wl.c2_circuit(22, nops=200, n_ry=5, h_qubits=12)]
    for c in circs:
        print(f"[case] {c.name} fused runs, group_items {items}", flush=True)
        outs = []
        # fuse every run (speculating at any size / never) / fuse none
        for opts in ({"fuse_runs": 4096, "speculate": 1, "speculate_group": 1},
                     {"fuse_runs": 4096, "speculate": 0, "speculate_group": 0},
                     {"fuse_runs": 0, "speculate": 0, "speculate_group": 0}):
            st = _gpu(abi, c, opts=dict(opts, group_items=items))
            outs.append(st.export() + (st.stats()["entries_updated"],))
            st.close()
        k0, a0, u0 = outs[-1]
        for k1, a1, u1 in outs[:-1]:
            assert np.array_equal(k1, k0)
            assert np.array_equal(a1.view(np.uint64), a0.view(np.uint64))
            assert u1 == u0                 # every op counted once on each path
        k1, a1, _ = outs[0]
        ora, _, _ = run_circuit(c)
        ok, _, oa = ora.export()
        compare(k1, a1, ok, oa, c.eps)


@pytest.mark.parametrize("form", ["chain", "fused"])
def test_capacity_failure_in_chain_or_fused_run(abi, form):
    """Capacity failure in a launch that carries a chain of one-target ops, or
    a one-target op with its following run: the state returns to the first
    op of the launch, failed_op names it, and resuming in a larger arena gives
    the oracle's result."""
    regs = [("a", 7 if form == "chain" else 8), ("b", 6), ("f", 1)]
    mk = wl.make_op
    if form == "chain":
        tail = [mk("RY", 1, qmask=1 << q, theta=0.3 + 0.2 * q) for q in range(3)]   # not a chain: targets differ
        body = [mk("RY", 2, qmask=1, theta=0.9), mk("RY", 2, qmask=1, theta=-0.4, ctls=[(0, 2, 1)]),
                mk("H", 2, qmask=1, ctls=[(0, 5, 0)])]
    else:
        tail = []
        body = [mk("RY", 2, qmask=1, theta=0.9), mk("ADD", 1, reg2=0), mk("XORC", 0, imm=0x2B),
                mk("X", 1, qmask=3, ctls=[(2, 0, 1)])]
    ops = wl.ops_array([mk("H", 0, qmask=(1 << regs[0][1]) - 1)] + tail + body + [mk("H", 0, qmask=0x01)])
    c = wl.Circuit(name=f"cap-{form}", regs=regs, ops=ops, eps=1e-14)
    print(f"[case] capacity failure in a {form} launch", flush=True)
    first = 1 + len(tail)                                  # index of the launch's first op
    st = abi.State(regs, eps=c.eps, cap_entries=1024 if form == "chain" else 256, table_bytes=0)
    n_before = 1024 if form == "chain" else 256
    assert st.capacity < 2 * n_before
    res = st.apply(ops, raise_on_error=False)
    assert res.status == abi.SS_E_CAPACITY and res.failed_op == first, (res.status, res.failed_op)
    gk, ga = st.export()
    ora, _, _ = run_circuit(c, ops=ops[:first])
    ok, _, oa = ora.export()
    s = compare(gk, ga, ok, oa, c.eps)
    assert s["n_gpu"] == n_before
    st.rebind(1 << 14)
    res = st.apply(ops[first:], raise_on_error=False)
    assert res.status == 0, abi.strerror(res.status)
    gk, ga = st.export()
    ora, _, _ = run_circuit(c)
    ok, _, oa = ora.export()
    compare(gk, ga, ok, oa, c.eps)
    st.close()


def test_c4_full_size_closed_form(abi):
    """The linear-solver walk at its full size (64 right-hand sides, 1024 rows
    x 8 slots, 200 steps, the bench's launch configuration: chained walk steps
    and fused runs) against its closed form for every entry: instance r, row
    rho, slot s, ancilla a has amplitude b_r[rho] c^3 [(R Ry(theta))^200 e0]_a,
    with theta = pi q16 / 2^15 from the table word and R = diag(i, -i)."""
    circ = wl.c4_batch(0, nrhs=64, steps=200)
    c0 = circ[0]
    print(f"[case] C4 full size: {len(circ)} right-hand sides, {len(c0.ops)} ops", flush=True)
    st = abi.State(c0.regs, ninst=len(circ), eps=c0.eps, cap_entries=1 << 22, table_bytes=1 << 16)
    st.load_qram(c0.tables[0])
    for i, c in enumerate(circ):
        st.set_entries(i, c.init_values, c.init_amps)
    st.apply(c0.ops)
    words = c0.tables[0].values.astype(np.int64)
    q = (words >> 16) & 0xFFFF
    q = np.where(q >= 0x8000, q - 0x10000, q).astype(np.float64)
    th = np.pi * q / 2.0 ** 15
    cth, sth = np.cos(th / 2), np.sin(th / 2)
    ry = np.stack([np.stack([cth, -sth], -1), np.stack([sth, cth], -1)], -2).astype(np.complex128)
    R = np.diag([1j, -1j])
    v = np.linalg.matrix_power(R @ ry, 200)[:, :, 0]          # (8192, 2): column e0
    addr = np.arange(8192, dtype=np.uint64)
    keys = np.concatenate([(addr << np.uint64(32)), (addr << np.uint64(32)) | np.uint64(1 << 45)])
    order = np.argsort(keys)
    for i in (0, 1, 31, 63):
        b = circ[i].init_amps
        amp = np.concatenate([b[addr >> np.uint64(3)] * C ** 3 * v[:, 0], b[addr >> np.uint64(3)] * C ** 3 * v[:, 1]])
        gk, ga = st.export(i)
        compare(gk, ga, keys[order].reshape(-1, 1), amp[order], c0.eps)
    assert st.nnz() <= 64 * 2 ** 14
    st.close()


def test_c3_full_size(abi):
    """The batching workload at its full size (1024 instances, caps 2^6..2^17,
    200..1000 ops each, capacity 2^28 entries) in the bench's configuration.
    Every instance against the oracle's stored result (tests/golden/
    c3_fingerprints.json, written by make_c3_fingerprints.py from the oracle
    alone): key set outside the band exact, four sampled amplitudes within
    1e-12, norm.  A spread of instances (the two largest caps with the
    shortest op lists, two of the next size, the median and the three
    smallest) against the oracle run live beside the GPU, entry by entry."""
    import json
    import os
    from multiprocessing import get_context

    from oracle_pool import oracle_export
    from parity import check_fingerprint, compare_arrays
    from paper_2503_15118_amd import batch
    golden = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "c3_fingerprints.json")))
    fps = golden["instances"]
    circ = wl.c3_batch(0, ninst=1024)
    assert len(fps) == len(circ) and all(fp["inst"] == i for i, fp in enumerate(fps))
    caps = sorted({c.cap_bits for c in circ})
    by_cost = sorted(range(len(circ)), key=lambda i: fps[i]["oracle_s"])
    spread = [i for i in by_cost if circ[i].cap_bits == caps[-1]][:2]
    spread += [i for i in by_cost if circ[i].cap_bits == caps[-2]][:2]
    order = sorted(range(len(circ)), key=lambda i: (circ[i].cap_bits, i))
    spread += [order[len(order) // 2]] + order[:3]
    print(f"[case] C3 full size: {len(circ)} instances, live oracle on {spread}", flush=True)
    with get_context("spawn").Pool(len(spread)) as pool:
        pending = pool.map_async(oracle_export, [circ[i] for i in spread])
        st, res = batch.run_batched(circ, cap_entries=1 << 28, table_bytes=0)
        assert res.status == 0
        exports = [st.export(i) for i in range(len(circ))]
        st.close()
        for i, (gk, ga) in enumerate(exports):
            check_fingerprint(gk, ga, circ[i].eps, fps[i])
        print("[stats] every instance matches its stored oracle fingerprint", flush=True)
        live = pending.get(timeout=900)
    for i, (ok, oa) in zip(spread, live):
        gk, ga = exports[i]
        s = compare_arrays(gk, ga, ok, oa, circ[i].eps)
        print(f"[stats] instance {i} cap 2^{circ[i].cap_bits}: {s}", flush=True)


@pytest.mark.parametrize("eps", [1e-3, 1e-6, 1e-13, 0.0])
def test_chain_respects_prune_threshold(abi, eps):
    """Chained one-target ops prune once; the planner shortens chains so that
    the prunes left out cannot move an amplitude by more than 1e-12.  Ry then
    Ry where the first leaves a child of 5e-4 (pruned in between when eps is
    1e-3), and longer chains of controlled and uncontrolled Ry / H."""
    theta1 = 2 * np.arcsin(5e-4)
    ops = [wl.make_op("H", 1, qmask=0b111), wl.make_op("RY", 0, qmask=1, theta=theta1),
           wl.make_op("RY", 0, qmask=1, theta=0.3)]
    rng = np.random.default_rng(3)
    for _ in range(14):
        ctl = [(1, int(rng.integers(0, 3)), int(rng.integers(0, 2)))] if rng.integers(0, 2) else []
        if rng.integers(0, 4) == 0:
            ops.append(wl.make_op("H", 0, qmask=1, ctls=ctl))
        else:
            ops.append(wl.make_op("RY", 0, qmask=1, theta=float(rng.uniform(-0.2, 0.2)), ctls=ctl))
    c = wl.Circuit(regs=[("q", 1), ("a", 3)], ops=wl.ops_array(ops), eps=eps, name=f"chain-eps{eps}")
    for chain in (1, 0):
        _check(abi, c, opts={"chain": chain})


def test_set_entries_rejects_duplicate_keys(abi):
    st = abi.State([("a", 4), ("b", 4)], cap_entries=1024)
    vals = np.array([[1, 2], [3, 4], [1, 2 + 16]], dtype=np.uint64)   # the third truncates to the first
    amps = np.array([0.6, 0.8, 0.0], dtype=np.complex128)
    with pytest.raises(RuntimeError):
        st.set_entries(0, vals, amps)
    assert st.nnz() == 1                                      # unchanged: still |0>
    st.set_entries(0, vals[:2], amps[:2])
    k, a = st.export()
    assert k[:, 0].tolist() == [1 | (2 << 4), 3 | (4 << 4)]
    st.close()


def test_measure_fallback_matches_oracle(abi):
    """No running sum exceeds u*P (P subnormal, 0.99*P rounds to P): both
    sides take the largest field value with weight."""
    a = 1e-161
    vals = np.array([[2], [5]], dtype=np.uint64)
    amps = np.array([a, a], dtype=np.complex128)
    c = wl.Circuit(regs=[("x", 3)], ops=wl.ops_array([]), eps=0.0, init_values=vals, init_amps=amps)
    st = abi.state_for_circuit(c)
    ora = OracleState.from_circuit(c)
    assert st.measure(0, 0, 0.99) == ora.measure(0, 0.99) == (5, 0.5)
    st.close()
