"""Full-size parity of the HIP path (keys exact, amplitudes within 1e-12,
through the C ABI):

* the arithmetic-heavy circuit (2^20 -> 2^21 entries, 1001 ops) in the
  benchmark's launch configuration, every entry against its closed form
  (oracle/closed_forms.py, pinned against the map oracle);
* collapsing measurement on 2^21 and 2^20 entries (multi-tile probability
  scans over up to 2^20 distinct field values) against the closed form's
  marginals, and on an instance > 0 of a batched state against the oracle;
* keys of four 64-bit words (W = 4) over several tiles through permutation,
  sort, group and expansion kernels, with and without grouping.
"""
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


def test_c2_full_size_every_entry(abi):
    """Every one of the 2^21 entries of the arithmetic-heavy circuit (seed 0,
    the benchmark's input and options) against the closed form."""
    c = wl.c2_circuit(0)
    print(f"[case] {c.name} full size, every entry", flush=True)
    st = abi.state_for_circuit(c, cap_entries=1 << 22)
    st.apply(c.ops)
    gk, ga = st.export()
    ck, ca = c2_closed_form(c)
    s = compare_arrays(gk, ga, ck, ca, c.eps)
    assert s["n_gpu"] == s["n_oracle"] == s["shared"] == 2 ** 21
    print("[stats]", s, flush=True)
    st.close()


def _marginal_outcome(keys, amps, word, shift, width, u):
    """The measurement reading: p(v) = sum of |a|^2 over entries with field v,
    P = sum of p(v) over ascending v, outcome = smallest v whose running sum
    exceeds u*P.  p(v) and P are summed with correct rounding (math.fsum)
    where a sum has many terms.  Returns (v, p(v)/P, margin of u*P to the
    nearest running-sum boundary, mask of the entries with field v, p(v))."""
    import math
    vals = (keys[:, word] >> np.uint64(shift)) & np.uint64((1 << width) - 1)
    mag = amps.real ** 2 + amps.imag ** 2
    uv, inv = np.unique(vals, return_inverse=True)
    if len(uv) <= 16:
        p = np.array([math.fsum(mag[inv == j]) for j in range(len(uv))])
    else:
        p = np.bincount(inv, weights=mag)      # a few terms per value
    P = math.fsum(p)
    run = np.cumsum(p)
    j = int(np.searchsorted(run, u * P, side="right"))
    margin = float(np.min(np.abs(run - u * P)))
    return int(uv[j]), float(p[j] / P), margin, vals == uv[j], float(p[j])


def _prob_tol(n):
    """Rounding bound of the device's probability: per-tile sums of 256
    entries, then one sequential scan over the n/256 tile sums; relative
    error of p(v) and of P each at most (n/256 + 256) units of 2^-53."""
    return max(1e-12, 2.0 * (n / 256 + 256) * 2.0 ** -53)


def test_measure_large_states(abi):
    """Measure the flag over 2^21 entries, then register b over the 2^20
    survivors (about 2^20 distinct values), against the closed form."""
    c = wl.c2_circuit(5, nops=80, n_ry=2, h_qubits=20)
    print(f"[case] measure on {c.name}", flush=True)
    st = abi.state_for_circuit(c, cap_entries=1 << 22)
    st.apply(c.ops)
    ck, ca = c2_closed_form(c)
    gk, ga = st.export()
    compare_arrays(gk, ga, ck, ca, c.eps)
    assert len(gk) == 2 ** 21
    for reg, word, shift, width, us in ((3, 1, 32, 1, (0.3, 0.7)), (1, 0, 32, 32, np.linspace(0.05, 0.95, 19))):
        for u in us:
            v, prob, margin, keep, pv = _marginal_outcome(ck, ca, word, shift, width, float(u))
            if margin > 1e-8:
                break
        else:
            pytest.fail("no draw away from the running-sum boundaries")
        n = len(ck)
        gv, gp = st.measure(0, reg, float(u))
        assert gv == v, (gv, v)
        assert abs(gp - prob) <= _prob_tol(n), (gp, prob)
        ck, ca = ck[keep], ca[keep] / np.sqrt(pv)
        gk, ga = st.export()
        s = compare_arrays(gk, ga, ck, ca, c.eps)
        print(f"[stats] measured reg {reg}: v={v} p={prob:.3e} |dp|={abs(gp - prob):.1e} entries={s['n_gpu']}",
              flush=True)
    st.close()


def test_measure_batched_instance(abi):
    """Collapsing measurement of one instance (> 0) of a batched state: that
    instance equals the oracle after its measurement, the others are
    untouched."""
    from paper_2503_15118_amd import batch
    circ = wl.c3_batch(4, ninst=6, lo_bits=8.0, hi_bits=12.0, len_lo=60, len_hi=120)
    st, res = batch.run_batched(circ, cap_entries=1 << 18)
    oras = [run_circuit(c)[0] for c in circ]
    for inst, reg, u in ((3, 0, 0.41), (5, 2, 0.77), (1, 1, 0.18)):
        print(f"[case] measure instance {inst} register {reg}", flush=True)
        gv, gp = st.measure(inst, reg, u)
        ov, op = oras[inst].measure(reg, u)
        assert gv == ov and abs(gp - op) <= 1e-12
        for i, c in enumerate(circ):
            gk, ga = st.export(i)
            ok, _, oa = oras[i].export()
            compare(gk, ga, ok, oa, c.eps)
    st.close()


def _w4_circuit(seed, h=12):
    """Registers of 40, 40, 60, 60 qubits and a flag: keys of four words.
    H on h qubits of a, then arithmetic, controlled X (one or two controls),
    Ry on the flag (some controlled) and two H on a qubit of b or d once it
    varies (sorted or grouped merges); 2^(h + 1) to 2^(h + 3) entries."""
    rng = np.random.default_rng(seed)
    regs = [("a", 40), ("b", 40), ("c", 60), ("d", 60), ("flag", 1)]
    widths = [w for _, w in regs]
    qa = rng.choice(40, size=h, replace=False)
    ops = [wl.make_op("H", 0, qmask=int(sum(1 << int(q) for q in qa)))]
    hpos = set(int(x) for x in rng.choice(np.arange(20, 90), size=2, replace=False))
    for i in range(90):
        if i in hpos:
            r = 1 + 2 * int(rng.integers(0, 2))
            ops.append(wl.make_op("H", r, qmask=1 << int(rng.integers(0, widths[r]))))
            continue
        k = int(rng.integers(0, 8))
        if k == 0:
            d, s = (int(x) for x in rng.choice(4, size=2, replace=False))
            ops.append(wl.make_op("ADD", d, reg2=s))
        elif k == 1:
            d, s = (int(x) for x in rng.choice(4, size=2, replace=False))
            ops.append(wl.make_op("SUB", d, reg2=s))
        elif k == 2:
            d = int(rng.integers(0, 4))
            ops.append(wl.make_op("MULC", d, imm=int(rng.integers(0, 1 << 62)) | 1))
        elif k == 3:
            d, s = (int(x) for x in rng.choice(4, size=2, replace=False))
            ops.append(wl.make_op("XOR", d, reg2=s))
        elif k == 4:
            d = int(rng.integers(0, 4))
            ops.append(wl.make_op("XORC", d, imm=int(rng.integers(0, 1 << 62))))
        elif k == 5:
            r = [int(x) for x in rng.choice(4, size=2, replace=False)]
            ops.append(wl.make_op("X", r[0], qmask=1 << int(rng.integers(0, widths[r[0]])),
                                  ctls=[(r[1], int(rng.integers(0, widths[r[1]])), int(rng.integers(0, 2)))]))
        elif k == 6:
            ops.append(wl.make_op("RY", 4, qmask=1, theta=float(rng.uniform(0, 2 * np.pi)),
                                  ctls=[(3, int(rng.integers(0, 60)), 1)] if rng.integers(0, 2) else []))
        else:
            r = [int(x) for x in rng.choice(4, size=3, replace=False)]
            ops.append(wl.make_op("X", r[0], qmask=1 << int(rng.integers(0, widths[r[0]])),
                                  ctls=[(r[1], int(rng.integers(0, widths[r[1]])), 1),
                                        (r[2], int(rng.integers(0, widths[r[2]])), 0)]))
    return wl.Circuit(regs=regs, ops=wl.ops_array(ops), eps=1e-14, cap_bits=h + 3, name=f"w4-seed{seed}")


@pytest.mark.parametrize("grouping", [1, 0])
def test_four_word_keys_multi_tile(abi, grouping):
    c = _w4_circuit(1)
    print(f"[case] {c.name} grouping={grouping}", flush=True)
    st = abi.state_for_circuit(c, cap_entries=1 << 17)
    assert st.key_words == 4
    st.set_option("grouping", grouping)
    st.apply(c.ops)
    gk, ga = st.export()
    ora, _, _ = run_circuit(c)
    ok, _, oa = ora.export()
    s = compare_arrays(gk, ga, ok, oa, c.eps)
    assert s["n_oracle"] >= 2 ** 13, s
    print("[stats]", s, flush=True)
    st.close()
