"""Autotuner for the per-state launch options of the simulator.

Each option changes how one kernel category tiles its work, never what it
computes:

- ``perm_entries``: entries per lane of the key-permutation interpreter;
- ``group_items``: entries per lane of the interference (group / expand) kernels;
- ``pair_exchange``: how that launch finds partners in group mode (lane pairs or LDS);
- ``spec_items``: entries per lane of their speculative fixed-placement launch;
- ``sort_items``: entries per lane of a radix-sort scatter pass.

Because each option touches only its own category, the search is coordinate-wise:
for one option at a time, every value is tried with the others held at their
current best. It is scored by the HIP-event time of that option's categories over
a caller-supplied workload (``run(state)``), taking the median of a few trials;
a value replaces the current one only when it is faster by more than a margin
(5 %), so that run-to-run noise does not move the choice.
Results are cached in a JSON file keyed by (GPU arch, key words, log2 of the
entry count, batched or plain), so a later state of the same shape starts from
the tuned values (``Tuner.apply``).
"""
from __future__ import annotations

import json
import math
import os
import statistics
from typing import Callable, Dict, Iterable, Optional

SPACE: Dict[str, tuple] = {
    "perm_entries": (4, 8, 16),
    "group_items": (1, 2, 4),
    "pair_exchange": (0, 1, 2),
    "spec_items": (1, 2, 4, 8),
    "sort_items": (8, 16),
}
DEFAULTS: Dict[str, int] = {"perm_entries": 8, "group_items": 4, "pair_exchange": 2, "spec_items": 4,
                            "sort_items": 16}
CATEGORIES: Dict[str, tuple] = {
    "perm_entries": ("perm",),
    "group_items": ("group", "expand"),
    "pair_exchange": ("group",),
    "spec_items": ("group", "expand"),
    "sort_items": ("sort_pass",),
}


def default_cache_path() -> str:
    p = os.environ.get("SPARQS_TUNE_CACHE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "sparqs", "tune.json")


def device_arch(device="cuda:0") -> str:
    import torch
    name = getattr(torch.cuda.get_device_properties(torch.device(device)), "gcnArchName", "") or "unknown"
    return name.split(":")[0]


def bucket_key(arch: str, key_words: int, nnz: int, batched: bool) -> str:
    lg = int(round(math.log2(max(1, nnz))))
    return f"{arch}/W{key_words}/n{lg}/{'batched' if batched else 'plain'}"


class Tuner:
    def __init__(self, path: Optional[str] = None, trials: int = 3, margin: float = 0.05):
        self.path = path or default_cache_path()
        self.trials = int(trials)
        # a value replaces the current one only when faster by more than this
        # fraction: run-to-run noise then leaves the choice where it was
        self.margin = float(margin)
        self.cache: Dict[str, Dict[str, int]] = {}
        if os.path.exists(self.path):
            with open(self.path) as f:
                raw = json.load(f)
            for k, v in raw.items():
                opts = {o: int(v[o]) for o in SPACE if o in v and int(v[o]) in SPACE[o]}
                if opts:
                    self.cache[k] = opts

    def save(self):
        d = os.path.dirname(self.path)
        if d:
            os.makedirs(d, exist_ok=True)
        tmp = self.path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(self.cache, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)

    def lookup(self, key: str) -> Optional[Dict[str, int]]:
        """Options cached for `key`, else those of the nearest size bucket of
        the same arch, key width and mode, else None."""
        if key in self.cache:
            return dict(self.cache[key])
        head, _, tail = key.rpartition("/")
        base, _, nb = head.rpartition("/")
        try:
            lg = int(nb[1:])
        except ValueError:
            return None
        best, dist = None, None
        for k, v in self.cache.items():
            h2, _, t2 = k.rpartition("/")
            b2, _, n2 = h2.rpartition("/")
            if b2 != base or t2 != tail:
                continue
            try:
                d = abs(int(n2[1:]) - lg)
            except ValueError:
                continue
            if dist is None or d < dist:
                best, dist = v, d
        return dict(best) if best is not None else None

    def apply(self, state, key: str) -> Dict[str, int]:
        """Set the cached options (defaults where none) on `state`; returns them."""
        opts = dict(DEFAULTS)
        opts.update(self.lookup(key) or {})
        for k, v in opts.items():
            state.set_option(k, v)
        return opts

    def _score(self, state, run: Callable, cats: Iterable[str]) -> float:
        times = []
        for _ in range(self.trials):
            state.set_option("trace", 1)
            state.set_option("trace_reset", 1)
            run(state)
            tr = state.trace()
            state.set_option("trace", 0)
            times.append(sum(tr[c]["seconds"] for c in cats))
        return statistics.median(times)

    def tune(self, state, run: Callable, key: str, space: Optional[Dict[str, tuple]] = None,
             save: bool = True) -> Dict[str, int]:
        """Coordinate search over `space` (default: all options) on `state`.

        `run(state)` must apply the same workload each time (reset included) and
        leave every launch synchronised.  The winning options stay set on the
        state, are cached under `key` and returned.  An option whose categories
        never launched keeps its current value.
        """
        space = space or SPACE
        best = dict(DEFAULTS)
        best.update(self.lookup(key) or {})
        for k, v in best.items():
            state.set_option(k, v)
        run(state)                       # warm-up: code objects loaded, arena touched
        scores: Dict[str, Dict[int, float]] = {}
        for opt, values in space.items():
            cats = CATEGORIES[opt]
            res = {}
            for v in values:
                state.set_option(opt, v)
                res[v] = self._score(state, run, cats)
            scores[opt] = res
            if all(t == 0.0 for t in res.values()):
                state.set_option(opt, best[opt])
                continue
            cand = min(values, key=lambda x: (res[x], x != best[opt]))
            if best[opt] not in res or res[cand] < res[best[opt]] * (1.0 - self.margin):
                best[opt] = cand
            state.set_option(opt, best[opt])
        self.cache[key] = dict(best)
        self.last_scores = scores
        if save:
            self.save()
        return best
