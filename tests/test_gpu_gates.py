"""The rest of the gate and oracle set on the HIP path, against the oracle
(keys exact, amplitudes within 1e-12, through the C ABI): Y, Z, S, T and their
inverses, the phase gate, rotations by 2x2 complex matrices (diagonal and
off-diagonal ones keep each branch one branch; general ones interfere), add
a constant, multiply and divide; QFT-form circuits; complex rotations at full
size in the speculative and compacting one-target kernels."""
import numpy as np
import pytest

import workloads as wl
from oracle.closed_forms import c2_closed_form
from oracle.oracle import run_circuit
from parity import compare, compare_arrays

pytestmark = pytest.mark.gpu

ONE_TO_ONE = ("Y", "Z", "S", "SDG", "T", "TDG", "PHASE", "ADDC", "MUL", "DIV", "X", "REFLECT0")


@pytest.fixture(scope="module")
def abi():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2503_15118_amd import _abi
    return _abi


def _check(abi, c, opts=None, cap=None):
    print(f"[case] {c.name} nops={len(c.ops)} opts={opts}", flush=True)
    st = abi.state_for_circuit(c, cap_entries=cap)
    for k, v in (opts or {}).items():
        st.set_option(k, v)
    st.apply(c.ops)
    gk, ga = st.export()
    ora, _, _ = run_circuit(c)
    ok, _, oa = ora.export()
    s = compare(gk, ga, ok, oa, c.eps)
    st.close()
    return s


@pytest.mark.parametrize("seed", range(6))
def test_one_to_one_kinds_bit_exact(abi, seed):
    """Gates that keep each branch one branch, and the arithmetic oracles, on
    imported superpositions: keys and amplitudes bit for bit (the products
    are formed in the oracle's order)."""
    c = wl.random_small_circuit(seed, kinds=ONE_TO_ONE, nops=80, with_init=True)
    s = _check(abi, c)
    assert s["bit_exact"] == s["shared"] == s["n_oracle"]


@pytest.mark.parametrize("seed", range(12))
def test_all_kinds_random_circuits(abi, seed):
    c = wl.random_small_circuit(seed + 40, kinds=wl.KINDS, nops=90, with_init=bool(seed % 2),
                                eps=(0.0 if seed % 4 == 3 else 1e-14))
    _check(abi, c)
    if seed < 4:
        _check(abi, c, opts={"grouping": 0})


def test_rotation_shapes(abi):
    """A diagonal and an off-diagonal rotation keep nnz (no interference
    launch); a general one groups, merges and prunes; controlled forms."""
    rng = np.random.default_rng(5)
    mats = [wl.random_unitary(rng, "diag"), wl.random_unitary(rng, "anti"), wl.random_unitary(rng)]
    ops = [wl.make_op("H", 0, qmask=0b1111), wl.make_op("ROT", 1, qmask=2, table=2, ctls=[(0, 1, 1)])]
    for t in (0, 1, 2, 0, 1):
        for q in range(3):
            ops.append(wl.make_op("ROT", 1, qmask=1 << q, table=t, ctls=[(0, q, 1)] if q % 2 else []))
    c = wl.Circuit(regs=[("a", 4), ("b", 3)], ops=wl.ops_array(ops), eps=1e-14, matrices=mats, name="rot-shapes")
    _check(abi, c)
    _check(abi, c, opts={"grouping": 0})


@pytest.mark.parametrize("n,x", [(6, 37), (12, 3001), (16, 40503)])
def test_qft_form(abi, n, x):
    """Textbook QFT of |x> (H and controlled phase gates, 2^n branches)."""
    for swaps in (False, True):
        _check(abi, wl.qft_circuit(n, x, swaps=swaps), cap=1 << (n + 1))


def test_qft_closed_form_multi_tile(abi):
    """QFT on 20 qubits: every one of the 2^20 amplitudes against
    2^-10 e^(2 pi i x rev(y) / 2^20)."""
    n, x = 20, 712345
    c = wl.qft_circuit(n, x)
    print(f"[case] {c.name}", flush=True)
    st = abi.state_for_circuit(c, cap_entries=1 << 21)
    st.apply(c.ops)
    gk, ga = st.export()
    y = np.arange(2 ** n, dtype=np.int64)
    rev = np.zeros_like(y)
    for b in range(n):
        rev |= ((y >> b) & 1) << (n - 1 - b)
    expect = np.exp(2j * np.pi * ((x * rev) % 2 ** n) / 2 ** n) / 2 ** (n / 2)
    s = compare_arrays(gk, ga, y.astype(np.uint64).reshape(-1, 1), expect, c.eps, atol=1e-12)
    assert s["shared"] == 2 ** n
    st.close()


@pytest.mark.parametrize("seed", [0, 1])
def test_complex_rotation_full_size(abi, seed):
    """The arithmetic-heavy circuit with complex rotations on the flag
    (2^20 -> 2^21 entries, 1001 ops; grouped pairs take the speculative
    fixed-placement launch first), every entry against the closed form."""
    c = wl.c2_rot_circuit(seed)
    print(f"[case] {c.name} full size", flush=True)
    st = abi.state_for_circuit(c, cap_entries=1 << 22)
    st.apply(c.ops)
    gk, ga = st.export()
    ck, ca = c2_closed_form(c)
    s = compare_arrays(gk, ga, ck, ca, c.eps)
    assert s["shared"] == 2 ** 21
    print("[stats]", s, flush=True)
    st.close()


def test_batched_all_kinds(abi):
    """Per-instance op lists with every kind (shared table and matrices)."""
    from paper_2503_15118_amd import batch
    base = wl.random_small_circuit(3, kinds=wl.KINDS, nops=1)
    circ = []
    for i in range(6):
        c = wl.random_small_circuit(200 + i, kinds=wl.KINDS, nops=[40, 0, 65, 12, 51, 30][i])
        c.tables = base.tables
        c.matrices = base.matrices
        circ.append(c)
    print(f"[case] batched all kinds, {len(circ)} instances", flush=True)
    st, res = batch.run_batched(circ, cap_entries=1 << 16)
    for i, c in enumerate(circ):
        gk, ga = st.export(i)
        ora, _, _ = run_circuit(c)
        ok, _, oa = ora.export()
        compare(gk, ga, ok, oa, c.eps)
    st.close()


def test_invalid_new_ops_rejected(abi):
    st = abi.State([("a", 4), ("b", 4), ("c", 3), ("d", 3)], cap_entries=1024)
    good = st.load_matrix(np.array([[0, 1], [1, 0]], dtype=np.complex128))
    assert good == 0
    with pytest.raises(RuntimeError):
        st.load_matrix(np.array([[1, 1], [0, 1]], dtype=np.complex128))
    bad = [
        (wl.make_op("ROT", 0, qmask=0b11, table=0), abi.SS_E_ARG),        # more than one qubit
        (wl.make_op("ROT", 0, qmask=1, table=5), abi.SS_E_ARG),           # unknown matrix
        (wl.make_op("Z", 0, qmask=1 << 4), abi.SS_E_ARG),                 # qubit outside the register
        (wl.make_op("S", 0, qmask=1, ctls=[(0, 0, 1)]), abi.SS_E_ARG),    # control on the target
        (wl.make_op("MUL", 0, reg2=0, reg3=1), abi.SS_E_ARG),             # source == destination
        (wl.make_op("DIV", 0, reg2=1, reg3=2, reg4=0), abi.SS_E_ARG),     # quotient == remainder
        (wl.make_op("DIV", 0, reg2=1, reg3=2, reg4=3, ctls=[(3, 0, 1)]), abi.SS_E_ARG),  # control in remainder
        (wl.make_op("ADDC", 0, imm=3, ctls=[(0, 1, 1)]), abi.SS_E_ARG),   # control inside dst
    ]
    for op, code in bad:
        res = st.apply(abi.to_ss_ops(wl.ops_array([op])), raise_on_error=False)
        assert res.status == code, (op, res.status)
    assert st.nnz() == 1
    st.close()
