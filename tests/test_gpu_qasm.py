"""Circuits read by the OpenQASM 2.0 subset front end, run on the HIP path
(through the C ABI) against the oracle."""
import numpy as np
import pytest

from oracle.oracle import run_circuit
from paper_2503_15118_amd import qasm
from parity import compare
from test_qasm_pins import random_program

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def abi():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2503_15118_amd import _abi
    return _abi


@pytest.mark.parametrize("seed", range(6))
def test_random_programs(abi, seed):
    c = qasm.parse(random_program(seed + 100, nq=(7, 6), ngates=120)).circuit
    print(f"[case] qasm random program {seed}", flush=True)
    st = abi.state_for_circuit(c, cap_entries=1 << 14)
    st.apply(c.ops)
    gk, ga = st.export()
    ora, _, _ = run_circuit(c)
    ok, _, oa = ora.export()
    compare(gk, ga, ok, oa, c.eps)
    st.close()


def test_ghz_255_from_text(abi):
    n = 255
    text = "OPENQASM 2.0;\nqreg q[%d];\nh q[0];\n" % n + "".join(f"cx q[{i}], q[{i + 1}];\n" for i in range(n - 1))
    c = qasm.parse(text).circuit
    st = abi.state_for_circuit(c, cap_entries=1024)
    assert st.key_words == 4
    st.apply(c.ops)
    k, a = st.export()
    assert len(k) == 2 and np.all(a == 0.70710678118654752440)
    assert k[1].tolist() == [2 ** 64 - 1] * 3 + [2 ** 63 - 1]
    st.close()
