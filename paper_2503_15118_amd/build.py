"""Build the HIP library ``libsparqs.so`` for gfx950 (in-tree, no JIT).

The device code is split over several translation units (the planner and its
small kernels; the launchers of each large kernel family, the emitting ones
once per key width), compiled in parallel and linked into one library."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsparqs.so")
OBJ = os.path.join(HERE, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # FP64 amplitudes: every product and sum rounded on its own (no FMA
    # contraction), so interference results follow the plain definition.
    "-ffp-contract=off",
    # keep the compiler from emitting packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # Branches on wave-uniform values (the op interpreter's dispatch) stay
    # plain scalar branches.  Structurizing them makes every case region read
    # the dispatch's incoming key registers, which then interfere with the
    # merged results and cost a copy of every key register per op.
    "-mllvm", "-structurizecfg-skip-uniform-regions=true",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]

# (source, object name, extra defines)
UNITS = [("sparqs.hip", "sparqs", []), ("launch_sort.hip", "launch_sort", [])]
for _fam in ("pair", "spec", "multi", "perm"):
    for _w in (1, 2, 4):
        UNITS.append((f"launch_{_fam}.hip", f"launch_{_fam}_w{_w}", [f"-DSS_LW={_w}"]))


def _compile(unit, verbose):
    src, name, defs = unit
    obj = os.path.join(OBJ, name + ".o")
    cmd = [HIPCC] + FLAGS + defs + ["-I", os.path.join(ROOT, "include"), "-c", "-o", obj,
                                    os.path.join(CSRC, src)]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l)
    if out.strip():
        print(out, flush=True)
    if r.returncode:
        raise subprocess.CalledProcessError(r.returncode, cmd)
    return obj


def build(verbose: bool = True, jobs: int | None = None) -> str:
    os.makedirs(OBJ, exist_ok=True)
    jobs = jobs or min(len(UNITS), max(1, min(16, os.cpu_count() or 1)))
    with ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda u: _compile(u, verbose), UNITS))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-Wl,-z,defs", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
