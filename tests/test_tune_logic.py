"""Autotuner search and cache logic on the CPU, with a scripted state whose
per-category times depend on the options set on it."""
import json

from paper_2503_15118_amd import tune


class FakeState:
    """Times per category: perm favours 4 entries, group/expand favour 2 items,
    the sort favours 16 items; `calls` counts workload runs."""

    def __init__(self, perm_cost=None, group_cost=None, sort_cost=None):
        self.opts = {}
        self.tr = None
        self.calls = 0
        self.perm_cost = perm_cost or {4: 1.0, 8: 2.0, 16: 3.0}
        self.group_cost = group_cost or {1: 3.0, 2: 1.0, 4: 2.0}
        self.sort_cost = sort_cost or {8: 2.0, 16: 1.0}

    def set_option(self, k, v):
        if k == "trace_reset":
            self.tr = {c: {"seconds": 0.0} for c in ("perm", "sort_hist", "sort_pass", "group", "expand", "filter")}
            return
        self.opts[k] = v

    def trace(self):
        return self.tr

    def run(self, _st):
        self.calls += 1
        if self.tr is None or not self.opts.get("trace"):
            return
        self.tr["perm"]["seconds"] += self.perm_cost[self.opts["perm_entries"]]
        self.tr["group"]["seconds"] += self.group_cost[self.opts["group_items"]]
        self.tr["expand"]["seconds"] += 0.5 * self.group_cost[self.opts["group_items"]]
        self.tr["sort_pass"]["seconds"] += self.sort_cost[self.opts["sort_items"]]
        # an unrelated category must not influence the choice
        self.tr["filter"]["seconds"] += 10.0 * self.opts["perm_entries"]


def test_coordinate_search_picks_fastest_and_caches(tmp_path):
    path = str(tmp_path / "tune.json")
    t = tune.Tuner(path, trials=1)
    st = FakeState()
    key = tune.bucket_key("gfx950", 2, 1 << 21, False)
    assert key == "gfx950/W2/n21/plain"
    best = t.tune(st, st.run, key)
    # spec_items changes no time here: the default stays
    assert best == {"perm_entries": 4, "group_items": 2, "pair_exchange": 2, "spec_items": 4, "sort_items": 16}
    # the winners stay set on the state
    for k, v in best.items():
        assert st.opts[k] == v
    # one warm-up + one run per candidate value
    assert st.calls == 1 + sum(len(v) for v in tune.SPACE.values())
    raw = json.load(open(path))
    assert raw[key] == best
    # a fresh tuner reads the cache back; apply sets the options
    t2 = tune.Tuner(path)
    st2 = FakeState()
    assert t2.apply(st2, key) == best
    assert {k: st2.opts[k] for k in best} == best


def test_lookup_nearest_bucket_same_shape_only(tmp_path):
    t = tune.Tuner(str(tmp_path / "c.json"))
    t.cache = {
        "gfx950/W2/n21/plain": {"perm_entries": 4, "group_items": 2, "sort_items": 8},
        "gfx950/W2/n14/plain": {"perm_entries": 8, "group_items": 1, "sort_items": 8},
        "gfx950/W1/n20/plain": {"perm_entries": 8, "group_items": 4, "sort_items": 16},
        "gfx950/W2/n20/batched": {"perm_entries": 8, "group_items": 4, "sort_items": 16},
    }
    assert t.lookup("gfx950/W2/n22/plain")["group_items"] == 2
    assert t.lookup("gfx950/W2/n15/plain")["group_items"] == 1
    assert t.lookup("gfx950/W4/n20/plain") is None
    assert t.lookup("gfx942/W2/n21/plain") is None
    # defaults when nothing is cached
    st = FakeState()
    assert t.apply(st, "gfx950/W4/n20/plain") == tune.DEFAULTS


def test_ties_keep_current_value_and_idle_options_untouched(tmp_path):
    t = tune.Tuner(str(tmp_path / "c.json"), trials=1)
    st = FakeState(perm_cost={4: 1.0, 8: 1.0, 16: 1.0}, sort_cost={8: 0.0, 16: 0.0})
    best = t.tune(st, st.run, "gfx950/W1/n16/plain")
    assert best["perm_entries"] == tune.DEFAULTS["perm_entries"]   # tie: keep the default
    assert best["sort_items"] == tune.DEFAULTS["sort_items"]       # category never ran
    assert st.opts["sort_items"] == tune.DEFAULTS["sort_items"]


def test_corrupt_or_foreign_entries_are_ignored(tmp_path):
    path = tmp_path / "c.json"
    path.write_text(json.dumps({"k": {"perm_entries": 5, "group_items": 2, "bogus": 1}}))
    t = tune.Tuner(str(path))
    assert t.cache == {"k": {"group_items": 2}}


def test_margin_keeps_current_value_unless_clearly_faster(tmp_path):
    t = tune.Tuner(str(tmp_path / "c.json"), trials=1, margin=0.05)
    # 4 entries 3 % faster than the default 8: kept; 16 entries 10 % faster: taken
    st = FakeState(perm_cost={4: 0.97, 8: 1.0, 16: 1.5})
    assert t.tune(st, st.run, "gfx950/W2/n21/plain")["perm_entries"] == 8
    st = FakeState(perm_cost={4: 1.2, 8: 1.0, 16: 0.9})
    assert t.tune(st, st.run, "gfx950/W2/n22/plain")["perm_entries"] == 16
