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


def _mix64(x):
    """splitmix64 finaliser on a uint64 array (a fixed public bit mixer)."""
    x = np.asarray(x, dtype=np.uint64).copy()
    with np.errstate(over="ignore"):
        x ^= x >> np.uint64(30)
        x *= np.uint64(0xBF58476D1CE4E5B9)
        x ^= x >> np.uint64(27)
        x *= np.uint64(0x94D049BB133111EB)
        x ^= x >> np.uint64(31)
    return x


def fingerprint(keys, amps, eps, nsamp=4):
    """Compact summary of one exported state for stored expected values.

    keys: (n, W) uint64 in ascending order, amps: (n,) complex128.  Keys inside
    the band (|a| <= eps + BAND) are left out, as the comparison rule allows
    them to be missing.  Returns nnz outside the band, a hash of that key set,
    the amplitudes at the ``nsamp`` keys with the smallest mixed hash, the
    norm, and how many amplitudes lie within 1e-11 of the band edge (where the
    two sides could classify a key differently)."""
    import hashlib
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    amps = np.asarray(amps, dtype=np.complex128)
    band = eps + BAND
    mag = np.abs(amps)
    keep = mag > band
    k = keys[keep]
    a = amps[keep]
    h = hashlib.sha256(k.astype("<u8").tobytes()).hexdigest()[:32]
    mix = np.zeros(len(k), dtype=np.uint64)
    for w in range(k.shape[1]):
        mix = _mix64(mix ^ k[:, w])
    idx = np.argsort(mix, kind="stable")[:nsamp]
    samples = [[[int(x) for x in k[i]], float(a[i].real), float(a[i].imag)] for i in idx]
    return {"nnz": int(len(k)), "keyhash": h, "samples": samples,
            "norm": float(np.sum(mag * mag)), "near_band": int(np.sum(np.abs(mag - band) < 1e-11))}


def check_fingerprint(keys, amps, eps, fp, atol=1e-12):
    """Compare an exported state with a stored fingerprint (same rule as
    ``compare``: key set outside the band exact, sampled amplitudes within
    ``atol``)."""
    got = fingerprint(keys, amps, eps, nsamp=0)
    if fp["near_band"] == 0 and got["near_band"] == 0:
        assert got["nnz"] == fp["nnz"], (got["nnz"], fp["nnz"])
        assert got["keyhash"] == fp["keyhash"], "key set differs from the stored one"
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    for key, re, im in fp["samples"]:
        hit = np.all(keys[:, :len(key)] == np.array(key, dtype=np.uint64), axis=1)
        j = np.flatnonzero(hit)
        assert len(j) == 1, f"sampled key {key} missing"
        assert abs(amps[j[0]] - complex(re, im)) <= atol
    assert abs(got["norm"] - fp["norm"]) <= 1e-9
    return got


def _ascending(keys):
    """Rows strictly ascending as unsigned integers, word W-1 most significant."""
    if len(keys) < 2:
        return True
    lt = np.zeros(len(keys) - 1, dtype=bool)
    eq = np.ones(len(keys) - 1, dtype=bool)
    for w in range(keys.shape[1] - 1, -1, -1):
        a, b = keys[:-1, w], keys[1:, w]
        lt |= eq & (a < b)
        eq &= a == b
    return bool(np.all(lt))


def compare_arrays(gpu_keys, gpu_amps, ref_keys, ref_amps, eps, atol=1e-12):
    """``compare`` for large states, vectorised: the same rule, on (n, W)
    uint64 key arrays (both sides ascending)."""
    W = gpu_keys.shape[1]
    ref_keys = np.asarray(ref_keys, dtype=np.uint64)
    if ref_keys.shape[1] > W:
        assert np.all(ref_keys[:, W:] == 0), "reference key uses more words than the GPU layout"
        ref_keys = ref_keys[:, :W]
    assert _ascending(gpu_keys), "export is not strictly ascending"
    assert _ascending(ref_keys), "reference is not strictly ascending"

    def void(k):
        return np.ascontiguousarray(k[:, ::-1].astype(">u8")).view(f"V{8 * W}").ravel()

    gv, rv = void(gpu_keys), void(ref_keys)
    _, gi, ri = np.intersect1d(gv, rv, assume_unique=True, return_indices=True)
    only_g = np.ones(len(gv), dtype=bool)
    only_g[gi] = False
    only_r = np.ones(len(rv), dtype=bool)
    only_r[ri] = False
    band = eps + BAND
    bad_g = np.flatnonzero(only_g & (np.abs(gpu_amps) > band))
    bad_r = np.flatnonzero(only_r & (np.abs(ref_amps) > band))
    assert len(bad_g) == 0, f"{len(bad_g)} keys only on the GPU, e.g. {gpu_keys[bad_g[:3]].tolist()}"
    assert len(bad_r) == 0, f"{len(bad_r)} keys only in the reference, e.g. {ref_keys[bad_r[:3]].tolist()}"
    d = np.abs(gpu_amps[gi] - ref_amps[ri])
    err = float(d.max()) if len(d) else 0.0
    assert err <= atol, f"max amplitude error {err} > {atol}"
    return {"n_gpu": len(gv), "n_oracle": len(rv), "shared": len(gi), "max_err": err,
            "bit_exact": int(np.sum(gpu_amps[gi] == ref_amps[ri])),
            "band_only": int(only_g.sum() + only_r.sum())}
