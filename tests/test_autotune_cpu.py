"""Host logic of the autotuner: the coordinate search picks the fastest
measured candidate, measures each once, and the JSON cache round-trips."""
import types

from paper_1906_00874_amd import autotune as T


def test_search_picks_fastest_coordinate_wise():
    times = {(64, 0): 10.0, (48, 0): 8.0, (40, 0): 9.0, (32, 0): 12.0,
             (48, 192): 7.5, (48, 128): 9.5}
    seen = []

    def measure(w, k):
        seen.append((w, k))
        return times[(w, k)]

    best, table = T.search(measure)
    assert best == (48, 192)
    # widths at the default launch width, then launch widths at the best width
    assert seen == [(64, 0), (48, 0), (40, 0), (32, 0), (48, 192), (48, 128)]
    assert [(r["trunc_width"], r["workers"]) for r in table] == seen
    assert min(r["ms"] for r in table) == 7.5


def test_search_keeps_default_on_ties():
    best, _ = T.search(lambda w, k: 5.0)
    assert best == (64, 0)


def test_cache_round_trip(tmp_path):
    f = str(tmp_path / "tune.json")
    T._store(f, "a", {"trunc_width": 40, "workers": 0})
    T._store(f, "b", {"trunc_width": 64, "workers": 128})
    d = T._load(f)
    assert d["a"]["trunc_width"] == 40 and d["b"]["workers"] == 128


def test_signature_counts_sizes():
    p = types.SimpleNamespace(leaf_size=32, eta=2.0, eps_factor=1e-6, rank_cap_factor=32,
                              fixed_rank=0, precision=1)
    hs = [types.SimpleNamespace(n=n, params=p) for n in (1280, 5120, 1280)]
    s = T.signature(hs)
    assert s.startswith("n[1280x2,5120x1]-leaf32-eta2-eps1e-06-cap32-fix0-prec1")
