"""Benchmark: the sparse simulator hot path on one MI355X.

Workload (one "step"): the arithmetic-heavy sparse circuit -- registers a, b,
c of 32 qubits and a 1-qubit flag (97-bit key in two 64-bit words), H on 20
seeded qubits of a (2^20 branches), then 1000 seeded ops: register add/sub
mod 2^32, multiply by odd constants, XOR (register or constant), CNOT,
Toffoli and 10 Ry on the flag (2^21 branches from the first one).  Each step
resets the state to |0> and runs the whole op list through the C ABI.

value = sparse entries updated per second = (sum over ops of the entry count
the op reads) / wall time of the timed steps.  The dominant kernel's achieved
bandwidth comes from HIP events recorded around every launch on the state's
stream during the timed steps.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
import argparse
import contextlib
import gc
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, published peak



@contextlib.contextmanager
def no_gc():
    """Run a timed region without Python's cyclic garbage collector, as timeit
    does: a full collection of this process's heap (torch and numpy loaded,
    some 10^5 objects) takes tens of milliseconds on the host and would land
    in whichever timed step crosses its allocation threshold."""
    gc.collect()
    was = gc.isenabled()
    gc.disable()
    try:
        yield
    finally:
        if was:
            gc.enable()


def sources_sha():
    """Short hash of the kernel sources the committed counter summaries name."""
    import hashlib
    src = os.path.join(ROOT, "paper_2503_15118_amd", "csrc")
    return hashlib.sha256(open(os.path.join(src, "kernels.hip"), "rb").read()
                          + open(os.path.join(src, "kernels_common.hpp"), "rb").read()
                          + open(os.path.join(src, "sparqs_internal.h"), "rb").read()).hexdigest()[:16]


def counter_valu_busy(kernel_label):
    """Duration-weighted vector-pipe busy fraction of `kernel_label` from the
    committed SQ counter summary, or None when the kernel sources changed
    since the counters were taken or the summary is of another kernel."""
    path = os.path.join(ROOT, "profiles", "c2_perm_sq_counters.txt")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    if f"kernel sources sha256[:16] = {sources_sha()}" not in text or f"dispatch of {kernel_label};" not in text:
        return None
    for line in text.splitlines():
        if line.startswith("# over all rows: valu_busy (duration-weighted) = "):
            return float(line.rsplit("=", 1)[1])
    return None


def counter_traffic(kernel_label):
    """HBM bytes per launch of `kernel_label` from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary (scaled by a plain copy of known size),
    or None when the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "c2_hbm_counters.txt")
    if not os.path.exists(path) or kernel_label is None:
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    sha = sources_sha()
    if kv.get("sources_sha") != sha or ("traffic " + kernel_label) not in kv:
        return None
    return float(kv["traffic " + kernel_label])


def summarize_profile(pdir):
    """Write profiles/c2_kernel_stats.txt and profiles/c2_hbm_counters.txt
    from the CSV output of the rocprofv3 runs named in their headers
    (<pdir>/trace: --kernel-trace --stats; <pdir>/fetch, <pdir>/write: one
    --pmc counter each)."""
    import collections
    import csv
    sha = sources_sha()
    # the C2 part of the default run (the other sections launch the same
    # kernels at other sizes, which would mix into the averages)
    base = "python3 bench.py --no-cpu-baseline --calibrate-copy --sections ''"
    out = ["# rocprofv3 kernel statistics: arithmetic-heavy sparse circuit (97-bit key, 2^20 -> 2^21 entries, "
           "1001 ops)",
           "# command (from /tmp, TMPDIR=/tmp; bench.py's default run: autotuning, warm-up, entry count, timed "
           "steps, traced steps, graph replays):",
           f"#   rocprofv3 --kernel-trace --stats --output-format csv -d <dir>/trace -o c2 -- {base} --steps 5 "
           "--warmup 1",
           f"# summarised by: python3 bench.py --summarize-profile <dir>",
           f"# kernel sources sha256[:16] = {sha}",
           f'{"kernel":62s} {"calls":>6s} {"avg_us":>9s} {"total_ms":>9s} {"pct":>6s}']
    for r in csv.DictReader(open(os.path.join(pdir, "trace", "c2_kernel_stats.csv"))):
        name = r["Name"].split("(")[0][:62]
        out.append(f'{name:62s} {int(r["Calls"]):6d} {float(r["AverageNs"]) / 1e3:9.1f} '
                   f'{float(r["TotalDurationNs"]) / 1e6:9.3f} {float(r["Percentage"]):6.2f}')
    with open(os.path.join(ROOT, "profiles", "c2_kernel_stats.txt"), "w") as f:
        f.write("\n".join(out) + "\n")

    def agg(path):
        a = collections.defaultdict(list)
        for r in csv.DictReader(open(path)):
            a[r["Kernel_Name"].split("(")[0]].append(float(r["Counter_Value"]))
        return a
    fe = agg(os.path.join(pdir, "fetch", "c2_counter_collection.csv"))
    wr = agg(os.path.join(pdir, "write", "c2_counter_collection.csv"))
    # calibration: the 64 MiB device copy (the largest copyBuffer dispatch)
    copy_f, copy_w = max(fe["__amd_rocclr_copyBuffer"]), max(wr["__amd_rocclr_copyBuffer"])
    fs, ws = 65536.0 / copy_f, 65536.0 / copy_w
    pmc = f"{base} --steps 2 --warmup 0 --no-tune --graph-steps 0"
    lines = ["# HBM traffic from rocprofv3 PMC counters: arithmetic-heavy sparse circuit (97-bit key, "
             "2^20 -> 2^21 entries)",
             "# commands (from /tmp, TMPDIR=/tmp), one counter per run:",
             f"#   timeout -s KILL 120 rocprofv3 --pmc FETCH_SIZE --output-format csv -d <dir>/fetch -o c2 -- {pmc}",
             f"#   timeout -s KILL 120 rocprofv3 --pmc WRITE_SIZE --output-format csv -d <dir>/write -o c2 -- {pmc}",
             "# summarised by: python3 bench.py --summarize-profile <dir>",
             f"# kernel sources sha256[:16] = {sha}",
             "# calibration: --calibrate-copy runs one plain device copy of 64 MiB (65536 KiB read + 65536 KiB "
             "written)",
             f"#   copy FETCH_SIZE = {copy_f:.1f} KiB -> fetch_scale = {fs:.3f};  copy WRITE_SIZE = {copy_w:.1f} KiB "
             f"-> write_scale = {ws:.3f}",
             f'{"kernel":50s} {"n":>4s} {"FETCH_KiB":>11s} {"WRITE_KiB":>11s} {"scaled_MB":>10s}']
    for k in sorted(set(fe) | set(wr), key=lambda x: -sum(fe.get(x, [0]))):
        fv, wv = fe.get(k, [0]), wr.get(k, [0])
        af, aw = sum(fv) / len(fv), sum(wv) / len(wv)
        lines.append(f"{k[:50]:50s} {len(fv):4d} {af:11.1f} {aw:11.1f} {(af * fs + aw * ws) * 1024 / 1e6:10.2f}")
    lines.append("")
    for label in ("k_perm_fast<2, 8, false>", "k_perm_fast<2, 4, false>", "k_perm_fast<2, 16, false>",
                  "k_pair<2, 0, 4, false>", "k_pair<2, 1, 4, false>", "k_pair<2, 1, 4, true>",
                  "k_pair<2, 0, 2, false>", "k_pair<2, 1, 2, false>", "k_expand_slots<2, 5, 4>") + tuple(
                      "k_pair_spec<2, 0, %d, %s, %d>" % (i, r, x) for i in (1, 2, 4, 8) for r in ("false", "true")
                      for x in (0, 1, 2)):
        pk = "void sparqs::" + label
        if pk not in fe or pk not in wr:
            continue
        af, aw = sum(fe[pk]) / len(fe[pk]), sum(wr[pk]) / len(wr[pk])
        lines.append(f"traffic {label}: {(af * fs + aw * ws) * 1024:.0f}")
    lines += [f"fetch_scale: {fs:.4f}", f"write_scale: {ws:.4f}", f"sources_sha: {sha}"]
    with open(os.path.join(ROOT, "profiles", "c2_hbm_counters.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")
    sq = summarize_sq(pdir, base, sha) if os.path.isdir(os.path.join(pdir, "sq")) else []
    sm = summarize_sort_merge(pdir, sha) if os.path.isdir(os.path.join(pdir, "sm")) else []
    c3 = summarize_batched(pdir, sha) if os.path.isdir(os.path.join(pdir, "c3trace")) else []
    print("\n".join(out + lines + sq + sm + c3))


def summarize_batched(pdir, sha):
    """profiles/c3_batched_kernel_stats.txt: kernel statistics and HBM traffic
    of the batched run of the 1024-instance workload (<pdir>/c3trace:
    --kernel-trace --stats; <pdir>/c3fetch, <pdir>/c3write: one --pmc counter
    each, scaled by the 64 MiB calibration copy of the same run)."""
    import collections
    import csv
    run = ("python3 bench.py --workload c3 --no-plain --no-cpu-baseline --calibrate-copy --graph-steps 0")
    stats = {}
    for r in csv.DictReader(open(os.path.join(pdir, "c3trace", "c3_kernel_stats.csv"))):
        stats[r["Name"].split("(")[0].replace("void ", "")] = r

    def agg(path):
        a = collections.defaultdict(float)
        mx = collections.defaultdict(float)
        for r in csv.DictReader(open(path)):
            k = r["Kernel_Name"].split("(")[0].replace("void ", "")
            a[k] += float(r["Counter_Value"])
            mx[k] = max(mx[k], float(r["Counter_Value"]))
        return a, mx
    fe, fmx = agg(os.path.join(pdir, "c3fetch", "c3_counter_collection.csv"))
    wr, wmx = agg(os.path.join(pdir, "c3write", "c3_counter_collection.csv"))
    fs, ws = 65536.0 / fmx["__amd_rocclr_copyBuffer"], 65536.0 / wmx["__amd_rocclr_copyBuffer"]
    lines = ["# rocprofv3 kernel statistics and HBM traffic: batching workload (1024 C1-form instances, 30-bit "
             "key with the instance field, caps 2^6..2^18, 200..1000 ops), batched run only: the timed apply "
             "and the traced apply (kernel table) of the same op lists",
             "# commands (from /tmp, TMPDIR=/tmp):",
             f"#   rocprofv3 --kernel-trace --stats --output-format csv -d <dir>/c3trace -o c3 -- {run}",
             f"#   timeout -s KILL 240 rocprofv3 --pmc FETCH_SIZE --output-format csv -d <dir>/c3fetch -o c3 -- {run}",
             f"#   timeout -s KILL 240 rocprofv3 --pmc WRITE_SIZE --output-format csv -d <dir>/c3write -o c3 -- {run}",
             "# summarised by: python3 bench.py --summarize-profile <dir>",
             f"# kernel sources sha256[:16] = {sha}",
             f"# HBM bytes = FETCH_SIZE x {fs:.3f} + WRITE_SIZE x {ws:.3f} (KiB; scales from the 64 MiB copy of "
             "the same run), summed over the kernel's dispatches",
             f'{"kernel":40s} {"calls":>6s} {"avg_us":>9s} {"total_ms":>9s} {"read_GB":>8s} {"write_GB":>9s}']
    for name, r in sorted(stats.items(), key=lambda kv: -float(kv[1]["TotalDurationNs"])):
        if "sparqs::" not in name:
            continue
        lines.append(f'{name.replace("sparqs::", "")[:40]:40s} {int(r["Calls"]):6d} '
                     f'{float(r["AverageNs"]) / 1e3:9.1f} {float(r["TotalDurationNs"]) / 1e6:9.1f} '
                     f'{fe.get(name, 0.0) * fs * 1024 / 1e9:8.1f} {wr.get(name, 0.0) * ws * 1024 / 1e9:9.1f}')
    with open(os.path.join(ROOT, "profiles", "c3_batched_kernel_stats.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")
    return lines


def summarize_sort_merge(pdir, sha):
    """profiles/sort_merge_2e26_kernel_stats.txt: kernel statistics of the
    sort / merge section (<pdir>/sm: --kernel-trace --stats of that section
    alone), the radix-sort kernels and the merge launches at 2^26 entries."""
    import csv
    cmd = ("rocprofv3 --kernel-trace --stats --output-format csv -d <dir>/sm -o sm -- python3 bench.py "
           "--no-cpu-baseline --no-tune --steps 2 --warmup 1 --graph-steps 0 --sections sortmerge")
    lines = ["# rocprofv3 kernel statistics: sort and merge of 2^26 entries (2^25 random distinct keys, an H on an "
             "unused qubit, then the same H with grouping off: a sort of every entry on its idle bits and a merge "
             "of each pair), W = 1 (41-bit key) and W = 2 (97-bit key), three repetitions each; the run also "
             "steps the arithmetic-heavy circuit (small kernels of 2^21 entries mix into k_pair and the "
             "expansions)",
             "# command (from /tmp, TMPDIR=/tmp):",
             f"#   {cmd}",
             "# summarised by: python3 bench.py --summarize-profile <dir>",
             f"# kernel sources sha256[:16] = {sha}",
             f'{"kernel":62s} {"calls":>6s} {"avg_us":>9s} {"min_us":>9s} {"max_us":>9s} {"total_ms":>9s}']
    for r in csv.DictReader(open(os.path.join(pdir, "sm", "sm_kernel_stats.csv"))):
        name = r["Name"].split("(")[0][:62]
        if not any(k in name for k in ("k_sort", "k_pair<", "k_expand")):
            continue
        lines.append(f'{name:62s} {int(r["Calls"]):6d} {float(r["AverageNs"]) / 1e3:9.1f} '
                     f'{float(r["MinNs"]) / 1e3:9.1f} {float(r["MaxNs"]) / 1e3:9.1f} '
                     f'{float(r["TotalDurationNs"]) / 1e6:9.3f}')
    with open(os.path.join(ROOT, "profiles", "sort_merge_2e26_kernel_stats.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")
    return lines


def summarize_sq(pdir, base, sha):
    """profiles/c2_perm_sq_counters.txt: SQ instruction counters of every
    dispatch of the interpreter (<pdir>/sq: one --pmc run with
    --kernel-trace), durations joined by dispatch id."""
    import collections
    import csv
    cnt = collections.defaultdict(dict)
    names = {}
    for r in csv.DictReader(open(os.path.join(pdir, "sq", "sq_counter_collection.csv"))):
        d = int(r["Dispatch_Id"])
        cnt[d][r["Counter_Name"]] = float(r["Counter_Value"])
        names[d] = r["Kernel_Name"].split("(")[0]
    dur = {}
    for r in csv.DictReader(open(os.path.join(pdir, "sq", "sq_kernel_trace.csv"))):
        dur[int(r["Dispatch_Id"])] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
    # the kernel that runs the op interpreter longest: the permutation
    # launch, or a one-target launch with a fused run
    busy = collections.Counter()
    for d, n in names.items():
        if "k_perm_fast<" in n or ("k_pair_spec<" in n and ", true, " in n):
            busy[n] += dur.get(d, 0.0)
    if not busy:
        return []
    kname = busy.most_common(1)[0][0]
    label = kname.replace("void sparqs::", "")
    counters = "SQ_INSTS_VALU SQ_INSTS_SALU SQ_INSTS_LDS SQ_INSTS_BRANCH SQ_WAVES SQ_WAVE_CYCLES SQ_BUSY_CYCLES " \
               "SQ_INSTS_SMEM"
    lines = ["# SQ instruction counters of the permutation-run interpreter: arithmetic-heavy sparse circuit "
             "(97-bit key, 2^21 entries)",
             "# command (from /tmp, TMPDIR=/tmp):",
             f"#   timeout -s KILL 150 rocprofv3 --pmc {counters} --kernel-trace --output-format csv -d <dir>/sq "
             f"-o sq -- {base} --no-tune --steps 2 --warmup 0 --graph-steps 0",
             "# summarised by: python3 bench.py --summarize-profile <dir>",
             f"# kernel sources sha256[:16] = {sha}",
             f"# one row per dispatch of {label}; instruction counts are wave instructions summed over the device",
             "# (waves: all waves of the grid, which is sized from an upper bound of the count, so some leave at once);",
             "# valu_busy = VALU x 4 cycles / 1024 SIMDs / (duration x 2.4 GHz)",
             f'{"dispatch":>8s} {"dur_us":>7s} {"waves":>7s} {"VALU":>10s} {"SALU":>10s} {"BRANCH":>10s} '
             f'{"LDS":>9s} {"SMEM":>8s} {"valu_busy":>9s}']
    tv = td = 0.0
    for d in sorted(k for k, n in names.items() if n == kname):
        c = cnt[d]
        t = dur.get(d, 0.0)
        busy = c.get("SQ_INSTS_VALU", 0.0) * 4 / 1024 / (t * 1e-6 * 2.4e9) if t > 0 else 0.0
        tv += c.get("SQ_INSTS_VALU", 0.0) * 4 / 1024 / 2.4e9
        td += t * 1e-6
        lines.append(f'{d:8d} {t:7.1f} {c.get("SQ_WAVES", 0):7.0f} {c.get("SQ_INSTS_VALU", 0):10.0f} '
                     f'{c.get("SQ_INSTS_SALU", 0):10.0f} '
                     f'{c.get("SQ_INSTS_BRANCH", 0):10.0f} {c.get("SQ_INSTS_LDS", 0):9.0f} '
                     f'{c.get("SQ_INSTS_SMEM", 0):8.0f} {busy:9.2f}')
    lines.append(f"# over all rows: valu_busy (duration-weighted) = {tv / td if td else 0.0:.2f}")
    with open(os.path.join(ROOT, "profiles", "c2_perm_sq_counters.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")
    return lines


def set_opts(st, opts):
    for kv in opts:
        k, v = kv.split("=", 1)
        st.set_option(k, int(v))


def host_info():
    """nproc and the CPU model of the host the oracle runs on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": len(os.sched_getaffinity(0)), "cpu_model": model}


def cpu_baseline(circ, nops_sample):
    """The oracle (std::map, one core) on a bounded sample of the same circuit:
    the H prelude and the first `nops_sample` ops after it."""
    from oracle.oracle import OracleState
    o = OracleState(circ.regs, circ.eps)
    s0, e0 = o.apply(circ.ops[:1])
    s1, e1 = o.apply(circ.ops[1:1 + nops_sample])
    sec, ent = s0 + s1, e0 + e1
    out = {"value": ent / sec, "unit": "entries/s", "cores": 1, "kind": "oracle",
           "sample": f"prelude H on 20 qubits + first {nops_sample} ops of the same circuit "
                     f"({ent} entry updates in {sec:.1f} s, std::map oracle, one thread)"}
    out.update(host_info())
    return out


def bench_batched(args, emit=True):
    """Batching: many C1-form instances (per-instance caps log-uniform in
    [2^6, 2^18], 200..1000 ops each) in one state, against the same instances
    run one at a time through the plain path on the same GPU."""
    import numpy as np
    import workloads as wl

    t0 = time.perf_counter()
    circ = wl.c3_batch(args.seed, ninst=args.ninst)
    gen_s = time.perf_counter() - t0
    # the oracle first: its worker processes fork before the GPU library loads
    cpu = None
    if not args.no_cpu_baseline:
        import dataclasses
        cpu = oracle_pool([dataclasses.replace(c, ops=c.ops[:150]) for c in circ[:16]],
                          "the first 150 ops of the first 16 instances of the batch")
    import torch
    from paper_2503_15118_amd import _abi, batch
    if args.calibrate_copy:
        calibration_copy()
    ops, off = batch.concat_ops(circ)
    zero = np.zeros((1, len(circ[0].regs)), dtype=np.uint64)
    one = np.array([1.0 + 0j])
    seq_s = None
    entries = None
    if not args.no_plain:
        # plain path, one instance at a time (apply calls timed)
        st = _abi.State(circ[0].regs, eps=circ[0].eps, cap_entries=1 << 20, table_bytes=0)
        seq_s = 0.0
        entries = 0
        plain_ops = [_abi.to_ss_ops(c.ops) for c in circ]
        st.apply(plain_ops[0])  # warm-up
        gc.collect()
        for c, o in zip(circ, plain_ops):
            st.set_entries(0, zero, one)
            e0 = st.stats()["entries_updated"]
            torch.cuda.synchronize()
            ta = time.perf_counter()
            st.apply(o)
            torch.cuda.synchronize()
            seq_s += time.perf_counter() - ta
            entries += st.stats()["entries_updated"] - e0
        st.close()
    # batched
    cap = 1 << args.batch_cap_log2
    bs = batch.batch_state(circ, cap_entries=cap, table_bytes=0)
    set_opts(bs, args.opt)
    s0 = bs.stats()
    with no_gc():
        torch.cuda.synchronize()
        tb = time.perf_counter()
        res = bs.apply(ops, inst_offsets=off)
        torch.cuda.synchronize()
        bat_s = time.perf_counter() - tb
    stats = {k: v - s0[k] for k, v in bs.stats().items()}
    nnz_b = bs.nnz()
    if entries is None:
        entries = stats["entries_updated"]
    # the same batch replayed from a captured HIP graph (captured once from
    # |0> in every instance; the replay starts from the same state)
    graph = None
    if args.graph_steps != 0:
        for i in range(len(circ)):
            bs.set_entries(i, zero, one)
        g = bs.capture(ops, inst_offsets=off)
        for i in range(len(circ)):
            bs.set_entries(i, zero, one)
        with no_gc():
            torch.cuda.synchronize()
            tg = time.perf_counter()
            g.launch()
            torch.cuda.synchronize()
            graph_s = time.perf_counter() - tg
        assert bs.nnz() == nnz_b
        g.close()
        graph = {"batched_graph_s": graph_s, "batched_graph_entries_per_s": entries / graph_s}
        if seq_s is not None:
            graph["batched_graph_vs_plain"] = seq_s / graph_s
    # kernel table: the same batch again from |0>, with a HIP event pair
    # around every launch (not part of the timing above)
    for i in range(len(circ)):
        bs.set_entries(i, zero, one)
    bs.set_option("trace", 1)
    bs.apply(ops, inst_offsets=off)
    tr = bs.trace()
    bs.set_option("trace", 0)
    bs.close()
    out = {
        "workload": f"batching: {args.ninst} C1-form instances (20-bit key, caps 2^6..2^18 log-uniform, "
                    f"200..1000 ops), seed {args.seed}",
        "entries_updated": int(entries),
        "sequential_plain_s": seq_s,
        "batched_s": bat_s,
        "batched_vs_plain": seq_s / bat_s if seq_s else None,
        "sequential_entries_per_s": entries / seq_s if seq_s else None,
        "batched_entries_per_s": entries / bat_s,
        "final_nnz_sum": int(res.nnz),
        "rounds_sorts": stats["sorts"],
        "kernels": {k: {"launches": v["launches"], "ms": 1e3 * v["seconds"],
                        "GBps": v["bytes"] / v["seconds"] / 1e9 if v["seconds"] else None}
                    for k, v in tr.items() if v["launches"]},
        "generation_s": gen_s,
    }
    if graph is not None:
        out.update(graph)
    if cpu is not None:
        out["cpu_baseline"] = cpu
    if emit:
        print(json.dumps(out), flush=True)
    return out


def calibration_copy():
    """One plain device copy of 64 MiB: the reference the HBM counter
    summaries scale FETCH_SIZE and WRITE_SIZE by."""
    import torch
    src = torch.ones(64 << 20, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def _oracle_run(c):
    from oracle.oracle import OracleState
    o = OracleState.from_circuit(c)
    sec, ent = o.apply(c.ops)
    return sec, ent


def oracle_pool(circuits, what):
    """The oracle over host cores (one instance per process, forked before the
    GPU is touched): entries/s over the makespan, and per core."""
    import multiprocessing as mp
    workers = max(1, min(16, len(os.sched_getaffinity(0)), len(circuits)))
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(workers) as pool:
        res = pool.map(_oracle_run, circuits, chunksize=1)
    wall = time.perf_counter() - t0
    sec = sum(r[0] for r in res)
    ent = sum(r[1] for r in res)
    return {"value": ent / wall, "unit": "entries/s", "cores": workers, "kind": "oracle",
            "single_core_entries_per_s": ent / sec if sec > 0 else None,
            "sample": f"{what}: {len(circuits)} instances over {workers} processes, {ent} entry updates, "
                      f"makespan {wall:.2f} s, single-core sum {sec:.2f} s"}


def _kernel_table(tr, steps=1):
    return {k: {"launches": v["launches"] / steps, "avg_us": 1e6 * v["seconds"] / v["launches"],
                "ms_per_step": 1e3 * v["seconds"] / steps,
                "GBps": v["bytes"] / v["seconds"] / 1e9 if v["seconds"] else None}
            for k, v in tr.items() if v["launches"]}


def bench_c1(args):
    """Small circuits (20-bit keys, nnz <= 2^14, 300 ops): the latency-bound
    end.  Per seed: 2 warm-up runs, then the median of 10 timed runs."""
    import numpy as np
    import torch
    import workloads as wl
    from paper_2503_15118_amd import _abi

    seeds = list(range(args.c1_seeds))
    med, ents = [], []
    st = None
    for seed in seeds:
        c = wl.c1_circuit(seed)
        ops = _abi.to_ss_ops(c.ops)
        if st is None:
            st = _abi.State(c.regs, eps=c.eps, cap_entries=1 << 15, table_bytes=0)
        zero = np.zeros((1, len(c.regs)), dtype=np.uint64)
        one = np.array([1.0 + 0j])
        times = []
        for r in range(12):
            st.set_entries(0, zero, one)
            e0 = st.stats()["entries_updated"]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st.apply(ops)
            torch.cuda.synchronize()
            if r >= 2:
                times.append(time.perf_counter() - t0)
        ents.append(st.stats()["entries_updated"] - e0)
        med.append(float(np.median(times)))
    out = {"workload": f"C1-form circuits (a:7, b:7, anc:6; 300 ops; nnz <= 2^14), seeds 0..{len(seeds) - 1}",
           "median_us_per_circuit": 1e6 * float(np.median(med)),
           "max_us_per_circuit": 1e6 * float(np.max(med)),
           "entries_per_s": float(np.sum(ents) / np.sum(med))}
    if not args.no_cpu_baseline:
        from oracle.oracle import OracleState
        osec, oent = 0.0, 0
        for seed in seeds[:2]:
            c = wl.c1_circuit(seed)
            o = OracleState(c.regs, c.eps)
            sec, ent = o.apply(c.ops)
            osec += sec
            oent += ent
        out["cpu_baseline"] = {"value": oent / osec, "unit": "entries/s", "cores": 1, "kind": "oracle",
                               "sample": f"seeds 0..1 whole circuits ({oent} entry updates in {osec:.2f} s)"}
        out["gpu_vs_oracle"] = out["entries_per_s"] / out["cpu_baseline"]["value"]
    print(json.dumps(out), flush=True)


def bench_c4(args):
    """The linear-solver walk: 64 right-hand sides as instances of one state
    (52-bit key), each step QRAM load, 16 controlled Ry, unload, reflection."""
    import numpy as np
    import workloads as wl

    # the oracle first: its worker processes fork before the GPU library loads
    cpu = None
    if not args.no_cpu_baseline:
        cpu = oracle_pool(wl.c4_batch(args.seed, nrhs=8, steps=20),
                          "8 right-hand sides of the same matrix, 20 walk steps")
    import torch
    from paper_2503_15118_amd import _abi

    circ = wl.c4_batch(args.seed, nrhs=args.nrhs, steps=args.c4_steps)
    c0 = circ[0]
    ops = _abi.to_ss_ops(c0.ops)
    st = _abi.State(c0.regs, ninst=len(circ), eps=c0.eps, cap_entries=1 << 22, table_bytes=1 << 16)
    st.load_qram(c0.tables[0])
    set_opts(st, args.opt)

    def reset():
        for i, c in enumerate(circ):
            st.set_entries(i, c.init_values, c.init_amps)

    reset()
    st.apply(ops)   # warm-up
    times = []
    ent = 0
    for _ in range(args.c4_trials):
        reset()
        e0 = st.stats()["entries_updated"]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st.apply(ops)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        ent = st.stats()["entries_updated"] - e0
    # kernel table from one more batch with a HIP event pair around every launch
    reset()
    st.set_option("trace", 1)
    st.set_option("trace_reset", 1)
    st.apply(ops)
    tr = st.trace()
    st.set_option("trace", 0)
    kernels = _kernel_table(tr, 1)
    dom = max(kernels, key=lambda k: kernels[k]["ms_per_step"])
    out = {"workload": f"QRAM linear-solver walk: {len(circ)} right-hand sides (N=1024, 8 nnz/row), "
                       f"{args.c4_steps} steps, 52-bit key; seed {args.seed}",
           "ms_per_batch": 1e3 * float(np.median(times)), "entries_per_batch": int(ent),
           "entries_per_s": ent / float(np.median(times)), "nnz_final": st.nnz(),
           "kernels": kernels, "dominant": dom,
           "dominant_frac_of_8TBps": kernels[dom]["GBps"] / HBM_PEAK_GBS if kernels[dom]["GBps"] else None}
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


def bench_m6(args):
    """Roofline sweep: one op per launch on n random distinct keys, per op kind
    and size, timed with HIP events; algorithmic bytes per launch / time."""
    import numpy as np
    import workloads as wl
    from paper_2503_15118_amd import _abi

    rng = np.random.default_rng(args.seed)
    # a 1-qubit register that no key sets is the branching target
    layouts = {1: [("a", 20), ("b", 20), ("t", 1)], 2: [("a", 32), ("b", 32), ("c", 32), ("t", 1)]}
    rows = []

    def trace_rows(st, W, lg, kind, cats):
        tr = st.trace()
        for cat in cats:
            r = tr[cat]
            if r["launches"]:
                gbps = r["bytes"] / r["seconds"] / 1e9
                rows.append({"W": W, "log2_n": lg, "kind": kind if len(cats) == 1 else cat,
                             "launches": r["launches"], "avg_us": 1e6 * r["seconds"] / r["launches"],
                             "GBps": gbps, "frac_of_8TBps": gbps / HBM_PEAK_GBS})
                print(json.dumps(rows[-1]), file=sys.stderr, flush=True)

    def run(st, ops, reps=3, grouping_first=None):
        st.set_option("trace", 1)
        st.set_option("trace_reset", 1)
        for _ in range(reps):
            for i, o in enumerate(ops):
                if grouping_first is not None and i == 0:
                    st.set_option("grouping", grouping_first)
                st.apply(_abi.to_ss_ops(wl.ops_array([o])))
                st.set_option("grouping", 1)
        st.set_option("trace", 0)

    sizes = ([int(x) for x in args.m6_sizes.split(",")] if args.m6_sizes
             else list(range(args.m6_min_log2, args.m6_max_log2 + 1, 3)))
    for W, regs in layouts.items():
        for lg in sizes:
            n = 1 << lg
            w0, w1 = regs[0][1], regs[1][1]
            tb = (1 << 22) + 4096 if W == 1 else 4096
            st = _abi.State(regs, eps=1e-14, cap_entries=2 * n, table_bytes=tb)
            if W == 1:
                st.load_qram(wl.Table(values=rng.integers(0, 2 ** w1, size=2 ** w0, dtype=np.uint64),
                                      addr_bits=w0, word_bits=w1))
            hi = np.uint64(2 ** (w0 + w1) - 1) if w0 + w1 < 64 else np.uint64(2 ** 64 - 1)
            v = np.unique(rng.integers(0, hi, size=int(n * 1.1) + 16, dtype=np.uint64, endpoint=False))[:n]
            rng.shuffle(v)
            vals = np.zeros((len(v), len(regs)), dtype=np.uint64)
            vals[:, 0] = v & np.uint64((1 << w0) - 1)
            vals[:, 1] = v >> np.uint64(w0)
            amps = (rng.standard_normal(len(v)) + 1j * rng.standard_normal(len(v))) / np.sqrt(2 * len(v))
            st.set_entries(0, vals, amps)
            t = len(regs) - 1
            perm = [("X", wl.make_op("X", 0, qmask=1)),
                    ("ADD", wl.make_op("ADD", 1, reg2=0)),
                    ("MULC", wl.make_op("MULC", 0, imm=(0x9E3779B1 & ((1 << w0) - 1)) | 1)),
                    ("phase", wl.make_op("REFLECT0", 1))]
            if W == 1:
                perm.append(("QRAM", wl.make_op("QRAM_LOAD", 1, reg2=0, table=0)))
            for name, op in perm:
                run(st, [op], reps=1)              # warm-up
                run(st, [op])
                trace_rows(st, W, lg, name, ["perm"])
            h = wl.make_op("H", t, qmask=1)
            # H on t twice: an expansion (every key gets both children), then the
            # grouped merge of the adjacent pairs back to n entries
            run(st, [h, h], reps=1, grouping_first=0)
            run(st, [h, h], grouping_first=0)
            trace_rows(st, W, lg, "H", ["expand", "group"])
            # sort + merge on 2n entries where every idle key appears twice
            run(st, [h], reps=1)
            run(st, [h], reps=1, grouping_first=0)
            trace_rows(st, W, lg + 1, "sort", ["sort_hist", "sort_pass", "group"])
            st.close()
    # QRAM gathers from tables of 2^A 32-bit words at random addresses
    # (2^24 entries; bytes counted: key read and write, not the gathered word)
    for A in ([int(x) for x in args.m6_qram_bits.split(",")] if args.m6_qram_bits else []):
        n = 1 << 24
        # data in the low 32 bits, the address above it: both fields inside one
        # 32-bit half of the key, the interpreter's gather case
        regs = [("data", 32), ("addr", A)]
        st = _abi.State(regs, eps=1e-14, cap_entries=2 * n, table_bytes=(4 << A) + 4096)
        st.load_qram(wl.Table(values=rng.integers(0, 2 ** 32, size=2 ** A, dtype=np.uint64),
                              addr_bits=A, word_bits=32))
        v = np.unique(rng.integers(0, np.uint64(2 ** (A + 32) - 1), size=int(n * 1.1) + 16,
                                   dtype=np.uint64))[:n]
        rng.shuffle(v)
        vals = np.zeros((len(v), 2), dtype=np.uint64)
        vals[:, 0] = v & np.uint64(0xFFFFFFFF)
        vals[:, 1] = v >> np.uint64(32)
        st.set_entries(0, vals, np.full(len(v), 1.0 / np.sqrt(len(v)), dtype=np.complex128))
        op = wl.make_op("QRAM_LOAD", 0, reg2=1, table=0)
        run(st, [op], reps=1)
        run(st, [op])
        trace_rows(st, 1, 24, f"QRAM table 2^{A}", ["perm"])
        st.close()
    print(json.dumps({"workload": "roofline sweep: one op per launch on random distinct keys "
                                  "(W=1: a:20 b:20 t:1; W=2: a,b,c:32 t:1; QRAM: data:32 addr:A)",
                      "rows": rows}), flush=True)


def bench_sort_merge(args, lg=25):
    """Roofline of the sort and the merge: n = 2^lg random distinct keys, an H
    on an unused qubit doubles them to 2n = 2^(lg+1) entries, then the same H
    with grouping switched off sorts the 2n entries on their idle bits (every
    idle key twice) and merges each pair back to one entry.  Past the 256 MB
    last-level cache at these sizes.  Algorithmic bytes per launch / HIP-event
    time of the launch, against the 8 TB/s peak."""
    import numpy as np
    import workloads as wl
    from paper_2503_15118_amd import _abi
    layouts = {1: [("a", 20), ("b", 20), ("t", 1)], 2: [("a", 32), ("b", 32), ("c", 32), ("t", 1)]}
    n = 1 << lg
    out = {"entries_sorted": 2 * n, "rows": []}
    for W, regs in layouts.items():
        st = _abi.State(regs, eps=1e-14, cap_entries=2 * n, table_bytes=4096)
        set_opts(st, args.opt)
        i = np.arange(n, dtype=np.uint64)
        with np.errstate(over="ignore"):
            v = (i * np.uint64(0x9E3779B97F4A7C15 | 1)) & np.uint64((1 << 40) - 1)   # odd multiplier: distinct
            v ^= v >> np.uint64(17)
        vals = np.zeros((n, len(regs)), dtype=np.uint64)
        vals[:, 0] = v & np.uint64((1 << 20) - 1)
        vals[:, 1] = v >> np.uint64(20)
        if W == 2:
            vals[:, 2] = (i * np.uint64(2654435761)) & np.uint64(0xFFFFFFFF)
        st.set_entries(0, vals, np.full(n, 1.0 / np.sqrt(n), dtype=np.complex128))
        del vals, v, i
        t = len(regs) - 1
        h = _abi.to_ss_ops(wl.ops_array([wl.make_op("H", t, qmask=1)]))
        for rep in range(3):
            st.apply(h)                          # 2n entries (expansion)
            st.set_option("grouping", 0)
            if rep == 2:
                st.set_option("trace", 1)
                st.set_option("trace_reset", 1)
            st.apply(h)                          # sort 2n, merge to n
            st.set_option("trace", 0)
            st.set_option("grouping", 1)
        tr = st.trace()
        for cat, name in (("sort_hist", "k_sort_hist"), ("sort_pass", "k_sort_pass"), ("group", "merge (k_pair)")):
            r = tr[cat]
            if r["launches"]:
                gbps = r["bytes"] / r["seconds"] / 1e9
                out["rows"].append({"W": W, "kernel": name, "launches": r["launches"],
                                    "avg_us": 1e6 * r["seconds"] / r["launches"], "GBps": gbps,
                                    "frac": gbps / HBM_PEAK_GBS})
        st.close()
    return out


def bench_m7(args):
    """Stand-ins for the paper's benchmark circuits (textbook constructions with
    the printed qubit and branch counts): GHZ 23/40/255, QRAM 20 from one
    branch, swap test 25.  Per circuit: 2 warm-up runs, then the median of 10.
    The paper's CPU times (two 64-core Xeons; Table 1 one thread, Table 2 64
    threads) are printed beside them as context, not as a baseline."""
    import numpy as np
    import torch
    import workloads as wl
    from paper_2503_15118_amd import _abi

    paper = {"ghz23": (0.0005, 0.0006), "ghz40": (0.0006, 0.0005), "ghz255": (0.0006, 0.0008),
             "qram20": (1e-4, 0.4743), "swap_test25": (14.8518, 5.6675)}
    circuits = [("ghz23", wl.ghz_circuit(23)), ("ghz40", wl.ghz_circuit(40)), ("ghz255", wl.ghz_circuit(255)),
                ("qram20", wl.qram_circuit(1, 10, 10, superpose=False)), ("swap_test25", wl.swap_test_circuit(12))]
    rows = []
    for name, c in circuits:
        cap = 1 << 26 if name.startswith("swap") else 1 << 12
        st = _abi.state_for_circuit(c, cap_entries=cap)
        ops = _abi.to_ss_ops(c.ops)
        zero = np.zeros((1, len(c.regs)), dtype=np.uint64)
        one = np.array([1.0 + 0j])
        times = []
        for r in range(12):
            st.set_entries(0, zero, one)
            e0 = st.stats()["entries_updated"]
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st.apply(ops)
            torch.cuda.synchronize()
            if r >= 2:
                times.append(time.perf_counter() - t0)
        ent = st.stats()["entries_updated"] - e0
        row = {"circuit": name, "qubits": c.nqubits, "peak_branches": st.peak(), "final_branches": st.nnz(),
               "median_ms": 1e3 * float(np.median(times)), "entries_per_s": ent / float(np.median(times)),
               "paper_cpu_s_1_thread": paper[name][0], "paper_cpu_s_64_threads": paper[name][1]}
        if name.startswith("swap"):
            st.set_entries(0, zero, one)
            st.set_option("trace", 1)
            st.set_option("trace_reset", 1)
            st.apply(ops)
            row["kernels"] = _kernel_table(st.trace(), 1)
            st.set_option("trace", 0)
        st.close()
        rows.append(row)
        print(f"[m7] {name}: {row['median_ms']:.3f} ms", file=sys.stderr, flush=True)
    print(json.dumps({"workload": "paper benchmark stand-ins (GHZ, QRAM, swap test)", "rows": rows}), flush=True)


def _same_state(k1, a1, k0, a0, eps):
    """(within the comparison rule, bit-identical, max amplitude error) for two
    exports in ascending key order: keys with |a| > eps + 1e-9 on either side
    must appear on both; shared keys' amplitudes within 1e-12."""
    import numpy as np
    if len(k1) == len(k0) and np.array_equal(k1, k0):
        err = float(np.max(np.abs(a1 - a0))) if len(a1) else 0.0
        return err <= 1e-12, bool(np.array_equal(a1.view(np.uint64), a0.view(np.uint64))), err
    band = eps + 1e-9
    s1 = {tuple(int(x) for x in k): a for k, a in zip(k1, a1)}
    s0 = {tuple(int(x) for x in k): a for k, a in zip(k0, a0)}
    ok = all(k in s0 for k, a in s1.items() if abs(a) > band) and \
        all(k in s1 for k, a in s0.items() if abs(a) > band)
    shared = [k for k in s1 if k in s0]
    err = max((abs(s1[k] - s0[k]) for k in shared), default=0.0)
    return bool(ok and err <= 1e-12), False, float(err)


def bench_serving(args, emit=True):
    """Serving: a Poisson request stream mixing the four workload forms, served
    with footprint admission and continuous batching, against the same trace
    served one request at a time through the plain path."""
    import torch
    import workloads as wl
    from paper_2503_15118_amd import serve

    t0 = time.perf_counter()
    tr = wl.c5_trace(args.seed, rate=args.rate, duration=args.duration, hi_bits=args.serve_hi_bits,
                     c4_steps=args.c4_steps)
    gen_s = time.perf_counter() - t0

    def reqs():
        return [serve.Request(rid=i, arrival=t.arrival, kind=t.kind, circuits=t.circuits, peak=t.peak)
                for i, t in enumerate(tr)]

    free, total = torch.cuda.mem_get_info()
    budget = min(288 << 30, free) - (8 << 30)
    ex = serve.GpuExecutor()
    warm = reqs()[:4]
    for r in warm:
        r.arrival = 0.0
    serve.Server(ex, budget_bytes=budget, max_active=4, chunk_ops=args.chunk_ops).run(warm)
    srv = serve.Server(ex, budget_bytes=budget, max_active=args.slots, chunk_ops=args.chunk_ops)
    served = reqs()
    m = srv.run(served)
    seq_reqs = reqs()
    seq = serve.plain_sequential(seq_reqs, ex)
    # the first 50 requests: result in the mix against the same request served
    # alone (keys exactly equal outside the prune band, amplitudes within 1e-12)
    checked = within = ident = 0
    worst = 0.0
    alone = {r.rid: r for r in seq_reqs}
    for r in sorted((x for x in served if x.error is None), key=lambda x: x.rid)[:50]:
        checked += 1
        ok_all, id_all = True, True
        for inst, ((gk, ga), (ak, aa)) in enumerate(zip(r.result, alone[r.rid].result)):
            ok, ident_i, err = _same_state(gk, ga, ak, aa, r.circuits[inst].eps)
            ok_all, id_all, worst = ok_all and ok, id_all and ident_i, max(worst, err)
        within += int(ok_all)
        ident += int(id_all)
    kinds = {}
    for t in tr:
        kinds[t.kind] = kinds.get(t.kind, 0) + 1
    out = {
        "workload": f"serving: Poisson {args.rate:g} req/s for {args.duration:g} s, kinds uniform over "
                    f"C1..C4 forms, peak 2^8..2^{args.serve_hi_bits:g}, C4-form walk {args.c4_steps} steps; "
                    f"seed {args.seed}",
        "requests": len(tr), "kinds": kinds,
        "served": m, "sequential_plain": seq,
        "p50_ms": 1e3 * m["p50_s"], "p99_ms": 1e3 * m["p99_s"],
        "p99_vs_plain": seq["p99_s"] / m["p99_s"],
        "throughput_vs_plain": m["entries_per_s"] / seq["entries_per_s"],
        "slots": args.slots, "budget_bytes": budget, "generation_s": gen_s,
        "mix_vs_alone": {"checked": checked, "within_rule": within, "bit_identical": ident,
                         "max_abs_amp_err": worst},
    }
    if emit:
        print(json.dumps(out), flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-ops", type=int, default=16)
    ap.add_argument("--grouping", type=int, default=1, help="0: sort before every interference op")
    ap.add_argument("--group-items", type=int, default=4)
    ap.add_argument("--sort-items", type=int, default=16)
    ap.add_argument("--perm-entries", type=int, default=8)
    ap.add_argument("--spec-items", type=int, default=8)
    ap.add_argument("--pair-exchange", type=int, default=2)
    ap.add_argument("--tile-order", type=int, default=1)
    ap.add_argument("--opt", action="append", default=[], metavar="KEY=VALUE",
                    help="extra ss_set_option on the state (c2, c4)")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep --group-items/--sort-items/--perm-entries instead of autotuning them")
    ap.add_argument("--tune-cache", default=None, help="autotuner JSON cache (default: per-user cache)")
    ap.add_argument("--graph-steps", type=int, default=None,
                    help="also time this many steps replayed from a captured HIP graph (default: --steps; 0: off)")
    ap.add_argument("--no-plain", action="store_true",
                    help="c3: batched run only, without the one-at-a-time plain path it is compared with")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one plain 64 MiB device copy first (reference for HBM counters)")
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c3", "c4", "c5", "m6", "m7"])
    ap.add_argument("--sections", default="sortmerge,c3,c5",
                    help="with --workload c2 (the default), the other parts of the metric measured in the same "
                         "run and added to its JSON line ('' = none)")
    ap.add_argument("--c1-seeds", type=int, default=32)
    ap.add_argument("--nrhs", type=int, default=64)
    ap.add_argument("--c4-trials", type=int, default=3)
    ap.add_argument("--m6-min-log2", type=int, default=16)
    ap.add_argument("--m6-max-log2", type=int, default=25)
    ap.add_argument("--m6-sizes", default=None, help="comma-separated log2 sizes (overrides min/max)")
    ap.add_argument("--m6-qram-bits", default="16,20,24,28", help="QRAM table address widths to sweep ('' = none)")
    ap.add_argument("--rate", type=float, default=200.0)
    ap.add_argument("--duration", type=float, default=10.0)
    ap.add_argument("--serve-hi-bits", type=float, default=24.0)
    ap.add_argument("--c4-steps", type=int, default=200)
    ap.add_argument("--slots", type=int, default=8)
    ap.add_argument("--chunk-ops", type=int, default=256)
    ap.add_argument("--ninst", type=int, default=1024)
    ap.add_argument("--batch-cap-log2", type=int, default=28)
    ap.add_argument("--summarize-profile", default=None, metavar="DIR",
                    help="write the profiles/ summaries from rocprofv3 CSV output under DIR and exit")
    args = ap.parse_args()
    if args.summarize_profile:
        summarize_profile(args.summarize_profile)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "sharding is a design note, not an implemented path", file=sys.stderr)
        sys.exit(2)

    if args.workload == "c1":
        bench_c1(args)
        return
    if args.workload == "c3":
        bench_batched(args)
        return
    if args.workload == "c4":
        bench_c4(args)
        return
    if args.workload == "m6":
        bench_m6(args)
        return
    if args.workload == "m7":
        bench_m7(args)
        return
    if args.workload == "c5":
        bench_serving(args)
        return

    import numpy as np
    import torch
    import workloads as wl
    from paper_2503_15118_amd import _abi

    if args.calibrate_copy:
        calibration_copy()

    circ = wl.c2_circuit(args.seed)
    ops = _abi.to_ss_ops(circ.ops)
    st = _abi.State(circ.regs, eps=circ.eps, cap_entries=1 << 22, table_bytes=0)
    st.set_option("grouping", args.grouping)
    st.set_option("group_items", args.group_items)
    st.set_option("sort_items", args.sort_items)
    st.set_option("perm_entries", args.perm_entries)
    st.set_option("spec_items", args.spec_items)
    st.set_option("pair_exchange", args.pair_exchange)
    st.set_option("tile_order", args.tile_order)
    set_opts(st, args.opt)
    zero = np.zeros((1, len(circ.regs)), dtype=np.uint64)
    one = np.array([1.0 + 0j])

    def step():
        st.set_entries(0, zero, one)
        st.apply(ops)

    tuned = None
    if not args.no_tune:
        # one-time setup outside the timed region: coordinate search over the
        # per-category launch options, scored by their kernels' HIP-event time
        from paper_2503_15118_amd import tune
        tuner = tune.Tuner(args.tune_cache, trials=3)
        key = tune.bucket_key(tune.device_arch(), st.key_words, 1 << 21, False)

        def tune_run(_s):
            step()
            torch.cuda.synchronize()

        tuned = tuner.tune(st, tune_run, key)
        args.group_items = tuned["group_items"]
        args.sort_items = tuned["sort_items"]
        args.perm_entries = tuned["perm_entries"]
        args.spec_items = tuned["spec_items"]
        args.pair_exchange = tuned["pair_exchange"]

    for _ in range(args.warmup):
        step()
    s0 = st.stats()["entries_updated"]
    step()
    entries_per_step = st.stats()["entries_updated"] - s0
    nnz_final = st.nnz()

    # the timed region: K steps as a user runs them (no per-launch events)
    sy0 = st.stats()["host_syncs"]
    with no_gc():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        marks = []
        for _ in range(args.steps):
            step()
            # a step ends with the planner's own waits for the device, so the
            # host clock after it is close to the device's (a diagnostic only)
            marks.append(time.perf_counter())
        torch.cuda.synchronize()
        t1 = time.perf_counter()
    syncs = (st.stats()["host_syncs"] - sy0) / args.steps
    step_ms = np.diff(np.array([t0] + marks)) * 1e3

    # the roofline pass: the same K steps again with a HIP event pair around
    # every launch on the state's stream (the events themselves add host and
    # device time between launches, so `value` is not taken from this pass)
    st.set_option("trace", 1)
    st.set_option("trace_reset", 1)
    with no_gc():
        torch.cuda.synchronize()
        r0 = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        r1 = time.perf_counter()
    tr = st.trace()
    st.set_option("trace", 0)

    elapsed = t1 - t0
    value = entries_per_step * args.steps / elapsed

    # the same step with the circuit replayed from a captured HIP graph: one
    # host wait per replay instead of the planner's read-backs
    graph = None
    gsteps = args.steps if args.graph_steps is None else args.graph_steps
    if gsteps > 0:
        st.set_entries(0, zero, one)
        g = st.capture(ops)
        for _ in range(args.warmup):
            st.set_entries(0, zero, one)
            g.launch()
        s0 = st.stats()["entries_updated"]
        torch.cuda.synchronize()
        with no_gc():
            g0 = time.perf_counter()
            gmarks = []
            for _ in range(gsteps):
                st.set_entries(0, zero, one)
                g.launch()
                gmarks.append(time.perf_counter())
            torch.cuda.synchronize()
            g1 = time.perf_counter()
        gstep_ms = np.diff(np.array([g0] + gmarks)) * 1e3
        gent = (st.stats()["entries_updated"] - s0) / gsteps
        assert gent == entries_per_step, (gent, entries_per_step)
        assert st.nnz() == nnz_final
        graph = {"steps": gsteps, "ms_per_step": 1e3 * (g1 - g0) / gsteps,
                 "value": gent * gsteps / (g1 - g0),
                 "step_ms": {"median": float(np.median(gstep_ms)), "max": float(np.max(gstep_ms))}}
        g.close()
    kernels = {}
    for name, r in tr.items():
        if r["launches"] == 0:
            continue
        kernels[name] = {"launches_per_step": r["launches"] / args.steps,
                         "avg_us": 1e6 * r["seconds"] / r["launches"],
                         "ms_per_step": 1e3 * r["seconds"] / args.steps,
                         "GBps": r["bytes"] / r["seconds"] / 1e9 if r["seconds"] > 0 else None}
    dom = max(kernels, key=lambda k: kernels[k]["ms_per_step"])
    d = tr[dom]
    achieved = d["bytes"] / d["seconds"] / 1e9
    # the kernel behind each category at this configuration (W = 2 keys); the
    # Ry ops on grouped entries (2^21) take the speculative fixed placement
    # unless it is switched off, and the compacting launch after it then only
    # records the count
    optd = dict((kv.split("=", 1)[0], int(kv.split("=", 1)[1])) for kv in args.opt)
    spec_group = optd.get("speculate_group", 1 << 21)
    # the run of non-branching ops after each Ry goes into the Ry's launch
    fused = "true" if optd.get("fuse_runs", 4096) > 0 else "false"
    group_label = ("k_pair_spec<2, 0, %d, %s, %d>" % (args.spec_items, fused, args.pair_exchange)
                   if 0 < spec_group <= 1 << 21 else "k_pair<2, 0, %d, %s>" % (args.group_items, fused))
    label = {"perm": "k_perm_fast<2, %d, false>" % args.perm_entries,
             "group": group_label,
             "expand": "k_pair<2, 1, %d, false>" % args.group_items}.get(dom)
    traffic = counter_traffic(label)
    valu_busy = counter_valu_busy(label)
    gpu_kernel_ms = sum(k["ms_per_step"] for k in kernels.values())

    out = {
        "metric": "sparse entries updated/s + HBM GB/s; batched-vs-plain speedup; p99 latency",
        "value": value,
        "unit": "entries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "arithmetic-heavy sparse circuit: registers a,b,c (32 qubits) + flag, 97-bit key "
                        "in 2 words; H on 20 qubits of a, then 1000 ops (add/sub/mulc/xor/CNOT/Toffoli, "
                        "10 Ry on flag); nnz 2^20 -> 2^21; complex128; seed %d" % args.seed,
            "nnz_final": nnz_final,
            "ops": int(len(ops)),
            "entries_per_step": int(entries_per_step),
            "grouping": args.grouping,
            "group_items": args.group_items,
            "sort_items": args.sort_items,
            "perm_entries": args.perm_entries,
            "spec_items": args.spec_items,
            "pair_exchange": args.pair_exchange,
            "tile_order": args.tile_order,
            "autotuned": tuned is not None,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": dom,
            "kernel_name": label,
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            # the other side of the bound: the fraction of time the vector
            # pipe issues (SQ counters of the same kernel), well below 1 too:
            # the launch is limited by instruction issue (the op interpreter's
            # scalar dispatch) as much as by bytes
            "valu_busy": valu_busy,
            "issue_bound": True,
            "algorithmic_bytes_per_launch": d["bytes"] / d["launches"],
            "timing": "HIP event pair around every launch of the kernel on the state's stream, over a second "
                      "pass of the same steps right after the timed one",
            "limiter": {"perm": "instruction issue of the op interpreter, not HBM: the vector pipe is busy about "
                                "40 % of the time (SQ counters, profiles/c2_perm_sq_counters.txt)",
                        "group": "the fused run of non-branching ops (op interpreter, instruction issue: "
                                 "profiles/c2_perm_sq_counters.txt) on top of the HBM stream of the "
                                 "fixed-placement launch; a count-only launch follows it",
                        "expand": "HBM stream with compaction"}.get(dom),
        },
        "hbm_gbps": achieved,
        "gpu_kernel_ms_per_step": gpu_kernel_ms,
        "traced_ms_per_step": 1e3 * (r1 - r0) / args.steps,
        # host clock after every timed step (each ends with the planner's
        # waits): a single slow step shows up here as a max far above the median
        "timed_step_ms": {"median": float(np.median(step_ms)), "max": float(np.max(step_ms)),
                          "min": float(np.min(step_ms))},
        "host_syncs_per_step": syncs,
        "kernels": kernels,
        "graph_replay": graph,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(circ, args.cpu_ops)
    st.close()
    # the rest of the metric, same run: sort / merge roofline past the
    # last-level cache, batched against plain, served against plain
    secs = [x for x in args.sections.split(",") if x]
    if "sortmerge" in secs:
        out["roofline_sort_merge"] = bench_sort_merge(args)
        print(json.dumps({"section": "roofline_sort_merge", "done": True}), file=sys.stderr, flush=True)
    if "c3" in secs:
        b = bench_batched(args, emit=False)
        out["batched"] = {k: b[k] for k in ("workload", "sequential_plain_s", "batched_s", "batched_vs_plain",
                                            "sequential_entries_per_s", "batched_entries_per_s",
                                            "batched_graph_s", "batched_graph_vs_plain",
                                            "batched_graph_entries_per_s", "rounds_sorts", "kernels")
                          if k in b}
        print(json.dumps({"section": "batched", "done": True}), file=sys.stderr, flush=True)
    if "c5" in secs:
        sv = bench_serving(args, emit=False)
        out["serving"] = {k: sv[k] for k in ("workload", "requests", "p50_ms", "p99_ms", "p99_vs_plain",
                                             "throughput_vs_plain", "mix_vs_alone", "slots")}
        out["serving"]["served"] = sv["served"]
        out["serving"]["sequential_plain"] = sv["sequential_plain"]
        print(json.dumps({"section": "serving", "done": True}), file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
