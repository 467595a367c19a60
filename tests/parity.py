"""Comparison rule between the HIP path and the CPU oracle.

Keys outside the band B (|a| <= eps + 1e-9 on either side) must match exactly,
word for word; shared keys must agree within ``atol`` as a complex modulus;
keys inside B may be missing on one side.
"""
import numpy as np

BAND = 1e-9


def _key_tuples(keys, W):
    return [tuple(int(x) for x in row[:W]) for row in keys]


def compare(gpu_keys, gpu_amps, ora_keys, ora_amps, eps, atol=1e-12, W=None):
    """Returns a dict of statistics; raises AssertionError on a violation."""
    if W is None:
        W = gpu_keys.shape[1] if len(gpu_keys) else 1
    ok_ora = np.all(ora_keys[:, W:] == 0) if ora_keys.shape[1] > W else True
    assert ok_ora, "oracle key uses more words than the GPU layout"
    g = dict(zip(_key_tuples(gpu_keys, W), gpu_amps))
    o = dict(zip(_key_tuples(ora_keys, W), ora_amps))
    # GPU export must be strictly ascending (canonical order)
    gk = _key_tuples(gpu_keys, W)
    rev = [tuple(reversed(k)) for k in gk]
    assert all(rev[i] < rev[i + 1] for i in range(len(rev) - 1)), "export is not strictly ascending"
    band = eps + BAND
    only_g = [k for k in g if k not in o]
    only_o = [k for k in o if k not in g]
    bad_g = [k for k in only_g if abs(g[k]) > band]
    bad_o = [k for k in only_o if abs(o[k]) > band]
    assert not bad_g, f"{len(bad_g)} keys only on the GPU, e.g. {bad_g[:3]} amp {[g[k] for k in bad_g[:3]]}"
    assert not bad_o, f"{len(bad_o)} keys only in the oracle, e.g. {bad_o[:3]} amp {[o[k] for k in bad_o[:3]]}"
    shared = [k for k in g if k in o]
    err = max((abs(g[k] - o[k]) for k in shared), default=0.0)
    exact = sum(1 for k in shared if g[k] == o[k])
    assert err <= atol, f"max amplitude error {err} > {atol}"
    return {"n_gpu": len(g), "n_oracle": len(o), "shared": len(shared), "max_err": err,
            "bit_exact": exact, "band_only": len(only_g) + len(only_o)}
