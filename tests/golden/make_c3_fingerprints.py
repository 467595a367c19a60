"""Write tests/golden/c3_fingerprints.json: the oracle's result for every
instance of the 1024-instance batching workload (seed 0), summarised by
``tests.parity.fingerprint``.  Calls only the oracle (and the seeded input
generator); run from the repository root:

    python tests/golden/make_c3_fingerprints.py [--jobs N]
"""
import argparse
import json
import os
import sys
import time
from multiprocessing import get_context

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "tests"))

OUT = os.path.join(ROOT, "tests", "golden", "c3_fingerprints.json")


_CIRC = None


def one(i):
    global _CIRC
    import workloads as wl
    from oracle.oracle import run_circuit
    from parity import fingerprint
    if _CIRC is None:
        _CIRC = wl.c3_batch(0, ninst=1024)
    c = _CIRC[i]
    t = time.time()
    st, _, _ = run_circuit(c)
    k, _, a = st.export()
    fp = fingerprint(k[:, :1], a, c.eps)
    fp["inst"] = i
    fp["cap_bits"] = int(c.cap_bits)
    fp["nops"] = int(len(c.ops))
    fp["oracle_s"] = round(time.time() - t, 2)
    return fp


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=os.cpu_count() or 1)
    args = ap.parse_args()
    import workloads as wl
    from oracle import oracle
    oracle.build()
    circ = wl.c3_batch(0, ninst=1024)
    order = sorted(range(len(circ)), key=lambda i: -(circ[i].cap_bits * 10000 + len(circ[i].ops)))
    res = {}
    with get_context("spawn").Pool(args.jobs) as pool:
        for n, fp in enumerate(pool.imap_unordered(one, order)):
            res[fp["inst"]] = fp
            if n % 8 == 0:
                print(f"{n + 1}/{len(order)} done", flush=True)
    out = {"workload": "c3_batch(seed=0, ninst=1024)", "eps": circ[0].eps,
           "rule": "keys with |a| <= eps + 1e-9 left out; samples = 4 keys with the smallest splitmix64 hash",
           "instances": [res[i] for i in range(len(circ))]}
    with open(OUT, "w") as f:
        json.dump(out, f, separators=(",", ":"))
    print("wrote", OUT)


if __name__ == "__main__":
    main()
