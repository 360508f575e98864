"""The batch autotuner's persistent cache (host logic only): workload keys,
the JSON file, and that a cached class is planned without timing."""
import json

from paper_2203_03732_amd import autotune


def test_keys_bucket_shapes():
    k1 = autotune.cache_key("gfx950:sramecc+:xnack-", [100, 200, 300], 16, 0.05)
    k2 = autotune.cache_key("gfx950", [140, 220, 260], 16, 0.05)
    assert k1 == k2  # same arch, n_max bucket 512, mean bucket 256, batch bucket 4
    assert k1.startswith("gfx950|nmax512|nmean256|batch4|d16|")
    assert autotune.cache_key("gfx950", [100, 200, 300], 16, 0.01) != k1
    assert autotune.cache_key("gfx950", [100, 200, 300], 8, 0.05) != k1
    assert autotune.cache_key("gfx950", [100, 200, 300, 4], 16, 0.05) == k1  # still batch 4
    assert autotune.cache_key("gfx950", [100, 200, 600], 16, 0.05) != k1     # n_max 1024
    assert autotune.cache_key("gfx950", [100, 200, 300], 16, 0.05, origin="zero") != k1


def test_store_and_load_round_trip(tmp_path):
    path = str(tmp_path / "sub" / "tune.json")
    assert autotune.load(path) == {}
    autotune.store("a", {"engine": "lds", "team": 0, "cost_path": 0, "ms": 1.5}, path)
    autotune.store("b", {"engine": "teams", "team": 4, "cost_path": 1, "ms": 0.5}, path)
    data = autotune.load(path)
    assert data["a"]["engine"] == "lds" and data["b"]["team"] == 4
    with open(path) as fh:
        assert json.load(fh) == data
    (tmp_path / "bad.json").write_text("not json")
    assert autotune.load(str(tmp_path / "bad.json")) == {}


class _FakeCtx:
    device = 0

    def __init__(self):
        self.timed = 0
        self.planned = []

    def autotune_batch(self, ns, d, eps, X, Y, reps=3, eps_mode="algorithmic", origin="diag"):
        self.timed += 1
        return {"engine": "teams", "team": 2, "cost_path": 0}, 0.25, 11

    def batch(self, ns, d, eps, **kw):
        self.planned.append(kw["config"])
        return kw["config"]


def test_tuned_batch_times_once_per_class(tmp_path):
    path = str(tmp_path / "tune.json")
    ctx = _FakeCtx()
    cfg = autotune.tuned_batch(ctx, [100, 300], 16, 0.05, None, None, path=path, arch="gfx950")
    assert ctx.timed == 1 and cfg == {"engine": "teams", "team": 2, "cost_path": 0}
    entry = next(iter(autotune.load(path).values()))
    assert entry["ms"] == 0.25 and entry["tried"] == 11
    cfg2 = autotune.tuned_batch(ctx, [120, 290], 16, 0.05, None, None, path=path, arch="gfx950")
    assert ctx.timed == 1 and cfg2 == cfg  # same class: read from the cache
    autotune.tuned_batch(ctx, [1200, 290], 16, 0.05, None, None, path=path, arch="gfx950")
    assert ctx.timed == 2  # a new n_max bucket is timed
