"""GPU parity of the batched solver: every instance of a batch must be
bit-exact with the CPU oracle run on that instance alone (rounded costs from
the binary32 definition, matching, duals and statistics), and graph replays
must reproduce the direct run."""
import math

import numpy as np
import pytest

import oracle
from paper_2203_03732_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

STAT_KEYS = ("phases", "sum_free", "rounds", "max_rounds", "scanned",
             "matched_in_phases", "completed_pairs", "sum_k")


@pytest.fixture(scope="module")
def ctx():
    import paper_2203_03732_amd as prot
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = prot.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def pack(Xs):
    return torch.from_numpy(np.ascontiguousarray(np.concatenate(Xs, 0))).cuda()


def check_instances(ns, Xs, Ys, eps, out, stats, origin="diag", which=None, complete=True):
    mate_a, mate_b, y_a, y_b = (t.cpu().numpy() for t in out)
    offs = np.concatenate([[0], np.cumsum(ns)])
    idx = range(len(ns)) if which is None else which
    for i in idx:
        n, o = ns[i], offs[i]
        k, m = oracle.round_points_f32(Xs[i], Ys[i], eps)
        ref = oracle.solve_rounded(k, oracle.threshold(eps, n), origin=origin, complete=complete)
        for name, arr in (("mate_a", mate_a), ("mate_b", mate_b), ("y_a", y_a), ("y_b", y_b)):
            assert np.array_equal(arr[o:o + n], ref[name]), f"instance {i} (n={n}): {name}"
        for s in STAT_KEYS:
            assert stats[i][s] == ref["stats"][s], f"instance {i}: {s}"
        assert stats[i]["cost_scale"] == m
        if complete:
            d2 = ((Xs[i].astype(np.float64) - Ys[i].astype(np.float64)[ref["mate_b"]]) ** 2).sum(1)
            assert math.isclose(stats[i]["cost"], d2.sum() / m, rel_tol=1e-12)


@pytest.mark.parametrize("origin", ["diag", "zero"])
@pytest.mark.parametrize("d,eps", [(2, 0.05), (16, 0.05), (3, 0.1)])
def test_batched_small_bit_exact(ctx, d, eps, origin):
    rng = np.random.default_rng(d * 10 + int(eps * 100))
    ns = [1, 2, 7, 64] + [int(x) for x in rng.integers(8, 300, 12)]
    Xs = [rng.standard_normal((n, d)).astype(np.float32) for n in ns]
    Ys = [rng.standard_normal((n, d)).astype(np.float32) for n in ns]
    mate_a, mate_b, y_a, y_b, stats = ctx.solve_batched_points(ns, pack(Xs), pack(Ys), eps,
                                                               origin=origin)
    check_instances(ns, Xs, Ys, eps, (mate_a, mate_b, y_a, y_b), stats, origin)


def test_batched_matrix_core_build_bit_exact(ctx):
    """The matrix-core build of a batch (d >= 16) gives the same instances."""
    rng = np.random.default_rng(77)
    d, eps = 24, 0.05
    ns = [1, 5, 64, 65, 200, 333]
    Xs = [rng.standard_normal((n, d)).astype(np.float32) for n in ns]
    Ys = [(0.3 + rng.standard_normal((n, d))).astype(np.float32) for n in ns]
    ctx.set_cost_path("matrix_cores")
    try:
        out = ctx.solve_batched_points(ns, pack(Xs), pack(Ys), eps)
    finally:
        ctx.set_cost_path("auto")
    check_instances(ns, Xs, Ys, eps, out[:4], out[4])


def test_batched_matrix_core_build_shifted_gaussians(ctx):
    """Instances of the differentiable-loss workload's shape (n = 2048,
    d = 64, X ~ N(0, I), Y ~ N(0.5, I), eps = 0.01) built on the matrix cores
    and solved by teams: every instance equals the oracle's."""
    X, Y = synth.shifted_gaussian_batch(3, 2048, 64, 0.5, seed=5)
    ns = [2048] * 3
    Xs, Ys = list(X), list(Y)
    ctx.set_cost_path("matrix_cores")
    try:
        out = ctx.solve_batched_points(ns, pack(Xs), pack(Ys), 0.01)
    finally:
        ctx.set_cost_path("auto")
    check_instances(ns, Xs, Ys, 0.01, out[:4], out[4])


@pytest.mark.parametrize("origin", ["diag", "zero"])
def test_batched_teams_bit_exact(ctx, origin):
    """Instances above n = 1024 are solved by teams of phase-loop workgroups;
    every instance must still match the oracle, including uneven sizes."""
    rng = np.random.default_rng(11)
    ns = [2048, 1100, 1025, 64, 3, 1800]
    Xs = [rng.standard_normal((n, 8)).astype(np.float32) for n in ns]
    Ys = [(0.2 + rng.standard_normal((n, 8))).astype(np.float32) for n in ns]
    out = ctx.solve_batched_points(ns, pack(Xs), pack(Ys), 0.02, origin=origin)
    check_instances(ns, Xs, Ys, 0.02, out[:4], out[4], origin)


def test_batched_teams_partial_and_replay(ctx):
    """Teams honour max_phases and no completion, and a captured graph of a
    team batch replays to the direct result."""
    rng = np.random.default_rng(12)
    ns = [1500, 1200, 2000]
    Xs = [rng.random((n, 2), dtype=np.float32) for n in ns]
    Ys = [rng.random((n, 2), dtype=np.float32) for n in ns]
    X, Y = pack(Xs), pack(Ys)
    plan = ctx.batch(ns, 2, 0.01, max_phases=3, complete=False)
    plan.run(X, Y)
    torch.cuda.synchronize()
    direct = [t.clone() for t in (plan.mate_a, plan.mate_b, plan.y_a, plan.y_b)]
    st = plan.stats()
    mate_a, mate_b, y_a, y_b = (t.cpu().numpy() for t in direct)
    offs = np.concatenate([[0], np.cumsum(ns)])
    for i, n in enumerate(ns):
        k, _ = oracle.round_points_f32(Xs[i], Ys[i], 0.01)
        ref = oracle.solve_rounded(k, oracle.threshold(0.01, n), max_phases=3, complete=False)
        o = offs[i]
        for name, arr in (("mate_a", mate_a), ("mate_b", mate_b), ("y_a", y_a), ("y_b", y_b)):
            assert np.array_equal(arr[o:o + n], ref[name]), f"instance {i}: {name}"
        assert st[i]["phases"] == ref["stats"]["phases"]
        assert st[i]["status"] == (1 if ref["status"] == "partial" else 0)
    plan.capture(X, Y)
    for _ in range(3):
        for t in (plan.mate_a, plan.mate_b, plan.y_a, plan.y_b):
            t.fill_(-7)
        torch.cuda.synchronize()
        plan.replay()
        torch.cuda.synchronize()
        for a, b in zip((plan.mate_a, plan.mate_b, plan.y_a, plan.y_b), direct):
            assert torch.equal(a, b)
    plan.close()


def test_batched_large_instances(ctx):
    """Instances up to the batched limit (n = 2048) use the larger LDS layout."""
    rng = np.random.default_rng(3)
    ns = [2048, 1500, 1025, 33]
    Xs = [rng.random((n, 2), dtype=np.float32) for n in ns]
    Ys = [rng.random((n, 2), dtype=np.float32) for n in ns]
    out = ctx.solve_batched_points(ns, pack(Xs), pack(Ys), 0.02)
    check_instances(ns, Xs, Ys, 0.02, out[:4], out[4])


def test_batched_no_completion(ctx):
    rng = np.random.default_rng(4)
    ns = [100, 250, 31]
    Xs = [rng.standard_normal((n, 4)).astype(np.float32) for n in ns]
    Ys = [rng.standard_normal((n, 4)).astype(np.float32) for n in ns]
    out = ctx.solve_batched_points(ns, pack(Xs), pack(Ys), 0.1, complete=False)
    check_instances(ns, Xs, Ys, 0.1, out[:4], out[4], complete=False)


def test_minibatch_512_instances_d16_eps005(ctx):
    """512 instances, n uniform in [64, 1024], standard normal points in R^16,
    eps = 0.05: every instance bit-exact with the oracle."""
    ns, Xs, Ys = synth.gaussian_batch(512, 64, 1024, 16, seed=0)
    X, Y = pack(Xs), pack(Ys)
    b = ctx.batch(ns, 16, 0.05)
    b.run(X, Y)
    torch.cuda.synchronize()
    stats = b.stats()
    out = (b.mate_a, b.mate_b, b.y_a, b.y_b)
    check_instances(ns, Xs, Ys, 0.05, out, stats)
    b.close()


def test_graph_replay_matches_direct_run(ctx):
    rng = np.random.default_rng(8)
    ns = [int(x) for x in rng.integers(64, 700, 40)]
    Xs = [rng.standard_normal((n, 16)).astype(np.float32) for n in ns]
    Ys = [rng.standard_normal((n, 16)).astype(np.float32) for n in ns]
    X, Y = pack(Xs), pack(Ys)
    b = ctx.batch(ns, 16, 0.05)
    b.run(X, Y)
    torch.cuda.synchronize()
    ref = [t.clone() for t in (b.mate_a, b.mate_b, b.y_a, b.y_b)]
    ref_stats = b.stats()
    b.capture(X, Y)
    for rep in range(3):
        for t in (b.mate_a, b.mate_b, b.y_a, b.y_b):
            t.fill_(-7)
        b.stats_dev.zero_()
        torch.cuda.synchronize()
        b.replay()
        torch.cuda.synchronize()
        for got, want in zip((b.mate_a, b.mate_b, b.y_a, b.y_b), ref):
            assert torch.equal(got, want), f"replay {rep}"
        assert b.stats() == ref_stats
        # eager work between replays
        (X * 2.0).sum().item()
    b.close()


def test_batched_rejects_oversized_instance(ctx):
    import paper_2203_03732_amd as prot
    n = prot.load().prot_batch_max_n() + 1
    X = torch.zeros((n, 2), dtype=torch.float32, device="cuda")
    with pytest.raises(prot.ProtError) as e:
        ctx.solve_batched_points([n], X, X.clone(), 0.1)
    assert e.value.name == "unsupported"


@pytest.mark.parametrize("config", [{"engine": "lds"}, {"engine": "teams", "team": 2},
                                    {"engine": "teams", "team": 8},
                                    {"engine": "teams", "team": 0},
                                    {"engine": "lds", "cost_path": 1},
                                    {"engine": "teams", "team": 4, "cost_path": 1}])
def test_every_batch_configuration_gives_the_same_instances(ctx, config):
    """The configurations the autotuner chooses among (engine, team size,
    cost path) all give every instance exactly as the oracle."""
    rng = np.random.default_rng(5)
    d, eps = 16, 0.05
    ns = [1, 64, 300, 1024, 1025, 1500]
    Xs = [rng.standard_normal((n, d)).astype(np.float32) for n in ns]
    Ys = [rng.standard_normal((n, d)).astype(np.float32) for n in ns]
    plan = ctx.batch(ns, d, eps, config=config)
    X, Y = pack(Xs), pack(Ys)
    plan.run(X, Y)
    torch.cuda.synchronize()
    check_instances(ns, Xs, Ys, eps, (plan.mate_a, plan.mate_b, plan.y_a, plan.y_b),
                    plan.stats())
    plan.close()


def test_batch_configuration_rejections(ctx):
    import paper_2203_03732_amd as prot
    with pytest.raises(prot.ProtError) as e:
        ctx.batch([1500, 20], 4, 0.1, config={"engine": "teams", "team": 1})  # needs 2
    assert e.value.name == "unsupported"
    with pytest.raises(prot.ProtError) as e:
        ctx.batch([10], 4, 0.1, config={"engine": "teams", "team": 9})
    assert e.value.name == "unsupported"
    with pytest.raises(prot.ProtError) as e:
        ctx.batch([10], 4, 0.1, config={"engine": "lds", "cost_path": 5})
    assert e.value.name == "arg"


def test_autotuner_picks_a_configuration_and_caches_it(ctx, tmp_path):
    from paper_2203_03732_amd import autotune
    rng = np.random.default_rng(9)
    d, eps = 16, 0.05
    ns = [int(x) for x in rng.integers(64, 700, 40)]
    Xs = [rng.standard_normal((n, d)).astype(np.float32) for n in ns]
    Ys = [rng.standard_normal((n, d)).astype(np.float32) for n in ns]
    X, Y = pack(Xs), pack(Ys)
    cfg, ms, tried = ctx.autotune_batch(ns, d, eps, X, Y, reps=2)
    assert tried >= 10 and ms > 0  # LDS + 8 team sizes, two cost paths
    assert cfg["engine"] in ("lds", "teams") and cfg["cost_path"] in (0, 1)
    path = str(tmp_path / "tune.json")
    plan = autotune.tuned_batch(ctx, ns, d, eps, X, Y, reps=1, path=path)
    entry = autotune.load(path)
    assert len(entry) == 1
    key = next(iter(entry))
    assert plan.config == {k: entry[key][k] for k in ("engine", "team", "cost_path")}
    plan.run(X, Y)
    torch.cuda.synchronize()
    check_instances(ns, Xs, Ys, eps, (plan.mate_a, plan.mate_b, plan.y_a, plan.y_b),
                    plan.stats(), which=[0, 7, 39])
    plan.close()
    # a second plan of the same class reads the cache and times nothing
    mtime = (tmp_path / "tune.json").stat().st_mtime_ns
    plan2 = autotune.tuned_batch(ctx, ns, d, eps, X, Y, reps=1, path=path)
    assert (tmp_path / "tune.json").stat().st_mtime_ns == mtime
    assert plan2.config == plan.config
    plan2.close()
