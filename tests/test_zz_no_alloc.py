"""The entry point for callers that cannot allocate (ss_create_state_noalloc):
a state whose scratch lives in the library's own device array gives the same
results as one created by ss_create_state, on two calls in a row (the second
with a smaller input, reusing the array), through the C ABI."""
import numpy as np
import pytest

import workloads as wl
from oracle.oracle import run_circuit
from parity import compare

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def abi():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2503_15118_amd import _abi
    return _abi


def _run(abi, c, cap, noalloc):
    st = abi.State(c.regs, eps=c.eps, cap_entries=cap, table_bytes=1 << 16, noalloc=noalloc)
    for t in c.tables:
        st.load_qram(t)
    if c.init_values is not None:
        st.set_entries(0, c.init_values, c.init_amps)
    st.apply(c.ops)
    k, a = st.export()
    nnz = st.nnz()
    st.close()
    return k, a, nnz


def test_noalloc_state_matches_arena_state(abi):
    cases = [(wl.c1_circuit(21), 1 << 16),                                 # larger input first
             (wl.random_small_circuit(5, nops=60, with_init=True), 1 << 10)]
    for c, cap in cases:
        print(f"[case] no-alloc state vs arena state: {c.name} cap {cap}", flush=True)
        k0, a0, n0 = _run(abi, c, cap, noalloc=False)
        k1, a1, n1 = _run(abi, c, cap, noalloc=True)
        assert n0 == n1 == len(k1)
        assert np.array_equal(k0, k1) and np.array_equal(a0.view(np.uint64), a1.view(np.uint64))
        ora, _, _ = run_circuit(c)
        ok, _, oa = ora.export()
        compare(k1, a1, ok, oa, c.eps)


def test_noalloc_one_state_per_gpu(abi):
    c = wl.random_small_circuit(6, nops=10)
    st = abi.State(c.regs, eps=c.eps, cap_entries=1 << 10, table_bytes=1 << 16, noalloc=True)
    with pytest.raises(RuntimeError):
        abi.State(c.regs, eps=c.eps, cap_entries=1 << 10, table_bytes=1 << 16, noalloc=True)
    st.close()
    st2 = abi.State(c.regs, eps=c.eps, cap_entries=1 << 10, table_bytes=1 << 16, noalloc=True)
    assert st2.nnz() == 1
    st2.close()
