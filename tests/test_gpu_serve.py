"""Serving on the GPU: requests run concurrently (own streams, own arenas)
give the same results as each request alone and as the oracle."""
import numpy as np
import pytest

import workloads as wl
from oracle.oracle import run_circuit
from parity import compare

pytestmark = pytest.mark.gpu


def _requests(tr):
    from paper_2503_15118_amd import serve
    return [serve.Request(rid=i, arrival=t.arrival, kind=t.kind, circuits=t.circuits, peak=t.peak)
            for i, t in enumerate(tr)]


def _run_alone(ex, r):
    from paper_2503_15118_amd import serve
    h = ex.start(r, None)
    while not ex.step(h, 1 << 30):
        pass
    res, _ = ex.finish(h)
    ex.release(h)
    return res


def test_results_same_alone_and_in_mix():
    import torch
    from paper_2503_15118_amd import serve
    assert torch.cuda.is_available()
    tr = wl.c5_trace(7, rate=400.0, duration=0.06, hi_bits=14.0, c4_steps=3, c4_matrix_n=64)
    reqs = _requests(tr)
    print(f"[case] serving mix of {len(reqs)} requests: {[r.kind for r in reqs]}", flush=True)
    ex = serve.GpuExecutor()
    srv = serve.Server(ex, budget_bytes=8 << 30, max_active=4, chunk_ops=16)
    m = srv.run(reqs)
    assert m["completed"] == len(reqs), [r.error for r in srv.done if r.error]
    bit_identical = 0
    for r in srv.done:
        alone = _run_alone(ex, r)
        for inst, ((gk, ga), (ak, aa)) in enumerate(zip(r.result, alone)):
            c = r.circuits[inst]
            compare(gk, ga, ak, aa, c.eps)
            bit_identical += int(np.array_equal(gk, ak) and np.array_equal(ga.view(np.uint64), aa.view(np.uint64)))
        if r.kind in ("c1", "c3"):
            ora, _, _ = run_circuit(r.circuits[0])
            ok, _, oa = ora.export()
            compare(r.result[0][0], r.result[0][1], ok, oa, r.circuits[0].eps)
    print(f"served {len(reqs)}; instances bit-identical alone vs mix: {bit_identical}", flush=True)


def test_mispredicted_footprint_pauses_and_resumes():
    from paper_2503_15118_amd import serve
    c = wl.c2_circuit(5, nops=200, n_ry=3, h_qubits=12)
    r = serve.Request(rid=0, arrival=0.0, kind="c2", circuits=[c], peak=1 << 10)   # 8x too small
    ex = serve.GpuExecutor()
    srv = serve.Server(ex, budget_bytes=4 << 30, max_active=2, chunk_ops=32)
    m = srv.run([r])
    assert m["completed"] == 1 and m["resumes"] >= 1
    ora, _, _ = run_circuit(c)
    ok, _, oa = ora.export()
    compare(r.result[0][0], r.result[0][1], ok, oa, c.eps)
