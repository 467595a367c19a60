"""QLSS building blocks on the HIP path (through the C ABI) against the
oracle: the block encoding U_A of a 32 x 32 matrix (controlled state
preparation from binary-tree angles read from QRAM, 32-bit angle words) and
walk steps R U_A, single states and all columns batched as instances."""
import numpy as np
import pytest

from oracle.oracle import run_circuit
from paper_2503_15118_amd.qlss import block_encoding, circuit, walk_step
from parity import compare

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def abi():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2503_15118_amd import _abi
    return _abi


def _matrix(seed, n, density=0.3):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((2 ** n, 2 ** n)) * (rng.random((2 ** n, 2 ** n)) < density)
    A[rng.integers(0, 2 ** n, 2 ** n), np.arange(2 ** n)] += 1.0
    return A


@pytest.mark.parametrize("steps", [0, 3])
def test_block_encoding_and_walk(abi, steps):
    A = _matrix(11, 5)
    be = block_encoding(A)
    ops = np.concatenate([be.ua] + [walk_step(be)] * steps)
    for j in (0, 17, 31):
        c = circuit(be, ops, j=j, name=f"qlss-n5-j{j}-steps{steps}")
        print(f"[case] {c.name} nops={len(ops)}", flush=True)
        st = abi.state_for_circuit(c, cap_entries=1 << 12)
        st.apply(ops)
        gk, ga = st.export()
        ora, _, _ = run_circuit(c)
        ok, _, oa = ora.export()
        compare(gk, ga, ok, oa, c.eps)
        if steps == 0:
            # top-left block: t = i, b = 0 (bits 37..41 of the key), d = a = 0
            top = ((gk[:, 0] >> np.uint64(37)) & np.uint64(31)) == 0
            col = np.zeros(32, dtype=np.complex128)
            col[(gk[top, 0] & np.uint64(31)).astype(np.int64)] = ga[top]
            assert np.max(np.abs(col - A[:, j] / np.linalg.norm(A))) < 2e-8
        st.close()


def test_walk_batched_over_columns(abi):
    """Every column j of A as its own instance in one state, 2 walk steps."""
    from paper_2503_15118_amd import batch
    A = _matrix(12, 4)
    be = block_encoding(A)
    ops = np.concatenate([be.ua, walk_step(be), walk_step(be)])
    circ = [circuit(be, ops, j=j, name=f"qlss-n4-col{j}") for j in range(16)]
    print(f"[case] batched walk, {len(circ)} instances, {len(ops)} ops", flush=True)
    st = batch.batch_state(circ, cap_entries=1 << 14, table_bytes=1 << 20)
    st.apply(ops)
    for i, c in enumerate(circ):
        gk, ga = st.export(i)
        ora, _, _ = run_circuit(c)
        ok, _, oa = ora.export()
        compare(gk, ga, ok, oa, c.eps)
    st.close()
