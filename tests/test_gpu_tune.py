"""The autotuner on the GPU: it picks valid options, and the tuned state gives
the same result (bit for bit) as the default options and matches the oracle."""
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


@pytest.mark.parametrize("form", ["c1", "c2"])
def test_tuned_options_valid_and_exact(abi, tmp_path, form):
    import torch
    from paper_2503_15118_amd import tune
    c = wl.c1_circuit(4) if form == "c1" else wl.c2_circuit(5, nops=120, n_ry=4, h_qubits=12)
    print(f"[case] tune {c.name}", flush=True)
    ops = abi.to_ss_ops(c.ops)
    st = abi.state_for_circuit(c)
    init_v = c.init_values if c.init_values is not None else np.zeros((1, len(c.regs)), dtype=np.uint64)
    init_a = c.init_amps if c.init_amps is not None else np.array([1.0 + 0j])

    def run(s):
        s.set_entries(0, init_v, init_a)
        s.apply(ops)
        torch.cuda.synchronize()

    t = tune.Tuner(str(tmp_path / "tune.json"), trials=2)
    key = tune.bucket_key(tune.device_arch(), st.key_words, 1 << (c.cap_bits or 14), False)
    best = t.tune(st, run, key)
    for k, v in best.items():
        assert v in tune.SPACE[k]
    run(st)
    k1, a1 = st.export()
    st.close()
    ref = abi.state_for_circuit(c)
    ref.apply(ops)
    k0, a0 = ref.export()
    ref.close()
    assert np.array_equal(k1, k0)
    assert np.array_equal(a1.view(np.uint64), a0.view(np.uint64))
    ora, _, _ = run_circuit(c)
    ok, _, oa = ora.export()
    compare(k1, a1, ok, oa, c.eps)
