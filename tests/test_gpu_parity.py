"""GPU parity: the HIP library, through its C ABI, against the CPU oracle.

Matchings, duals, statistics and the per-phase trace must be bit-exact given
the same rounded costs; the rounded costs themselves must be bit-exact with
the oracle's definitions (eq. (1) in binary64; the binary32 fma
squared-distance definition for point sets). Costs in binary64 agree to
rounding order (1e-12 relative)."""
import math

import numpy as np
import pytest

import oracle
from paper_2203_03732_amd import synth
from invariants import check_I1, check_I2, check_matching

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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.cpu().numpy()


def padded_k(k_np):
    """Device copy of an n x n int16 matrix in the library's pitched layout."""
    import paper_2203_03732_amd as prot
    n = k_np.shape[0]
    kp = np.full((n, prot.pitch(n)), 0x7FFF, np.int16)
    kp[:, :n] = k_np
    return dev(kp)


def assert_same(gpu, orc, what=""):
    for x in ("mate_a", "mate_b", "y_a", "y_b"):
        g = host(getattr(gpu, x))
        assert np.array_equal(g, orc[x]), f"{what}: {x} differs at {np.nonzero(g != orc[x])[0][:10]}"
    for s in STAT_KEYS:
        assert gpu.stats[s] == orc["stats"][s], f"{what}: stat {s} {gpu.stats[s]} != {orc['stats'][s]}"


# ----------------------------------------------------- rounded-cost builds

@pytest.mark.parametrize("n,eps", [(1, 0.1), (37, 0.1), (300, 0.01), (1000, 0.1), (777, 0.003)])
def test_round_costs_bit_exact(ctx, n, eps):
    C = synth.uniform_costs(n, seed=n)
    C[0, 0] = 1.0
    k = ctx.round_costs(dev(C), eps)
    torch.cuda.synchronize()
    kg = host(k)
    assert np.array_equal(kg[:, :n], oracle.round_cost(C, eps))
    assert (kg[:, n:] == 0x7FFF).all()


@pytest.mark.parametrize("n,d,storage", [(600, 2, "matrix"), (600, 3, "matrix"),
                                         (600, 2, "on_the_fly"), (20000, 2, "auto"),
                                         (20000, 3, "auto")])
@pytest.mark.parametrize("where", ["X", "Y"])
def test_points_reject_non_finite_then_recover(ctx, n, d, storage, where):
    """A NaN or an infinite coordinate (the plain maximum pass, the pruned one
    at n >= 16,384, either side) is refused; the solve after it, on clean
    points, starts from a cleared error word and equals the oracle."""
    import paper_2203_03732_amd as prot
    X, Y = synth.uniform_points(n, d, seed=n + d)
    for bad in (float("nan"), float("inf")):
        Xb, Yb = X.copy(), Y.copy()
        (Xb if where == "X" else Yb)[n // 3, d - 1] = bad
        with pytest.raises(prot.ProtError) as e:
            ctx.solve_points(dev(Xb), dev(Yb), 0.05, storage=storage)
        assert e.value.name == "range"
    gpu = ctx.solve_points(dev(X), dev(Y), 0.05, storage=storage)
    if n <= 1000:
        k, _ = oracle.round_points_f32(X, Y, 0.05)
        ref = oracle.solve_rounded(k, oracle.threshold(0.05, n))
        assert np.array_equal(host(gpu.mate_b), ref["mate_b"])
        assert np.array_equal(host(gpu.y_b), ref["y_b"])
    else:
        check_matching(host(gpu.mate_a), host(gpu.mate_b))


def test_points_enqueue_only(ctx):
    """Without statistics a point solve only enqueues: the status query
    reports how it ended, the outputs equal the oracle's, and a non-finite
    coordinate is reported by the status query."""
    import paper_2203_03732_amd as prot
    X, Y = synth.uniform_points(3000, 2, seed=40)
    res = ctx.solve_points(dev(X), dev(Y), 0.01, stats=False)
    assert res.stats == {}
    assert ctx.status() == "ok"
    k, _ = oracle.round_points_f32(X, Y, 0.01)
    orc = oracle.solve_rounded(k, oracle.threshold(0.01, 3000))
    for x in ("mate_a", "mate_b", "y_a", "y_b"):
        assert np.array_equal(host(getattr(res, x)), orc[x]), x
    Xb = X.copy()
    Xb[7, 1] = float("nan")
    ctx.solve_points(dev(Xb), dev(Y), 0.01, stats=False)
    with pytest.raises(prot.ProtError) as e:
        ctx.status()
    assert e.value.name == "range"
    res = ctx.solve_points(dev(X), dev(Y), 0.01)
    assert np.array_equal(host(res.mate_b), orc["mate_b"])


def test_round_costs_rejects_nan_and_range(ctx):
    import paper_2203_03732_amd as prot
    for bad in (float("nan"), -0.5, 1.5):
        C = synth.uniform_costs(64, seed=1)
        C[5, 7] = bad
        with pytest.raises(prot.ProtError) as e:
            ctx.round_costs(dev(C), 0.1)
        assert e.value.name == "range"
    with pytest.raises(prot.ProtError) as e:
        ctx.round_costs(dev(synth.uniform_costs(8)), 1.5)
    assert e.value.name == "eps"


@pytest.mark.parametrize("path", ["direct", "matrix_cores", "auto"])
@pytest.mark.parametrize("n,d,eps", [(1, 2, 0.1), (50, 2, 0.01), (1000, 2, 0.01),
                                     (513, 3, 0.005), (200, 5, 0.05), (300, 16, 0.05),
                                     (150, 17, 0.02), (130, 64, 0.01), (65, 4, 0.3),
                                     (700, 40, 0.01), (260, 96, 0.02)])
def test_build_costs_bit_exact(ctx, n, d, eps, path):
    X, Y = synth.uniform_points(n, d, seed=7 + d)
    ctx.set_cost_path(path)
    try:
        k, m = ctx.build_costs(dev(X), dev(Y), eps)
    finally:
        ctx.set_cost_path("auto")
    torch.cuda.synchronize()
    ko, mo = oracle.round_points_f32(X, Y, eps)
    assert float(host(m)[0]) == mo
    kg = host(k)
    assert np.array_equal(kg[:, :n], ko)
    assert (kg[:, n:] == 0x7FFF).all()


def test_build_costs_matrix_core_path_far_from_origin(ctx):
    """Points far from the origin make the matrix-core approximation's error
    bound large relative to the distances, so most entries take the exact
    fallback; the result must still equal the definition bit for bit."""
    rng = np.random.default_rng(12)
    n, d = 300, 24
    X = (100.0 + rng.standard_normal((n, d))).astype(np.float32)
    Y = (100.0 + rng.standard_normal((n, d))).astype(np.float32)
    for eps in (0.05, 0.003):
        ctx.set_cost_path("matrix_cores")
        try:
            k, m = ctx.build_costs(dev(X), dev(Y), eps)
        finally:
            ctx.set_cost_path("auto")
        torch.cuda.synchronize()
        ko, mo = oracle.round_points_f32(X, Y, eps)
        assert float(host(m)[0]) == mo
        assert np.array_equal(host(k)[:, :n], ko)


def test_build_costs_within_tolerance_of_binary64(ctx):
    """The binary32 cost is within 1e-5 of the binary64 cost (normalised),
    and every rounded-cost flip against binary64 is one step at a boundary."""
    n, eps = 700, 0.01
    X, Y = synth.uniform_points(n, 2, seed=3)
    k, m = ctx.build_costs(dev(X), dev(Y), eps)
    torch.cuda.synchronize()
    kg = host(k)[:, :n].astype(np.int64)
    c64, k64, m64 = oracle.points_cost_f64(X, Y, eps)
    assert abs(float(host(m)[0]) - m64) <= 1e-6 * m64
    assert np.abs(kg - k64).max() <= 1
    flips = kg != k64
    q = c64[flips] / eps
    assert np.all(np.abs(q - np.round(q)) < 1e-5 / eps)


# ------------------------------------------------------------ phase loop

CASES = [(1, 3, 0), (2, 1, 0), (7, 4, 1), (37, 9, 3), (100, 20, 5), (513, 15, 20),
         (1000, 30, 10), (1500, 7, 0)]


@pytest.mark.parametrize("origin", ["diag", "zero"])
@pytest.mark.parametrize("n,K,T", CASES)
def test_solve_rounded_bit_exact(ctx, n, K, T, origin):
    k = synth.random_k(n, K, seed=n * 31 + K)
    orc = oracle.solve_rounded(k, T, origin=origin, trace=True)
    gpu = ctx.solve_rounded(padded_k(k), T, n, origin=origin)
    assert gpu.status == "ok"
    assert_same(gpu, orc, f"n={n} K={K} T={T} {origin}")
    tr = ctx.trace()
    assert np.array_equal(tr, orc["trace"])


@pytest.mark.parametrize("origin", ["diag", "zero"])
def test_structured_instances(ctx, origin):
    n = 300
    cases = {"zeros": np.zeros((n, n), np.int16),
             "identity": np.where(np.eye(n, dtype=bool), 0, 9).astype(np.int16),
             "ramp": (np.add.outer(np.arange(n), np.arange(n)) % 13).astype(np.int16),
             "rows": np.repeat((np.arange(n) % 5)[:, None], n, 1).astype(np.int16),
             "cols": np.repeat((np.arange(n) % 5)[None, :], n, 0).astype(np.int16)}
    for name, k in cases.items():
        orc = oracle.solve_rounded(k, 2, origin=origin)
        gpu = ctx.solve_rounded(padded_k(k), 2, n, origin=origin)
        assert_same(gpu, orc, name)


def test_no_completion_and_invariants(ctx):
    n, K, T = 400, 25, 12
    k = synth.random_k(n, K, seed=5)
    orc = oracle.solve_rounded(k, T, complete=False)
    gpu = ctx.solve_rounded(padded_k(k), T, n, complete=False)
    assert_same(gpu, orc)
    check_matching(host(gpu.mate_a), host(gpu.mate_b))
    check_I1(host(gpu.mate_a), host(gpu.y_a), host(gpu.y_b))
    check_I2(k, host(gpu.mate_b), host(gpu.y_a), host(gpu.y_b))
    assert int((host(gpu.mate_b) < 0).sum()) <= T


def test_threshold_at_least_n(ctx):
    k = synth.random_k(50, 5, seed=2)
    gpu = ctx.solve_rounded(padded_k(k), 50, 50)
    orc = oracle.solve_rounded(k, 50)
    assert_same(gpu, orc)
    assert gpu.stats["phases"] == 0


def test_warm_start_phase_by_phase(ctx):
    """Resume on the GPU from the oracle's state after p phases, run one
    phase, and compare with the oracle after p + 1 phases."""
    n, K, T = 600, 12, 6
    k = synth.random_k(n, K, seed=77)
    kd = padded_k(k)
    full = oracle.solve_rounded(k, T, complete=False)
    state = None
    for p in range(full["stats"]["phases"]):
        ref = oracle.solve_rounded(k, T, max_phases=1, state=state, complete=False)
        st_dev = None if state is None else {x: dev(state[x]) for x in state}
        gpu = ctx.solve_rounded(kd, T, n, state=st_dev, max_phases=1, complete=False)
        assert gpu.status in ("partial", "ok")
        for x in ("mate_a", "mate_b", "y_a", "y_b"):
            assert np.array_equal(host(getattr(gpu, x)), ref[x]), f"phase {p}: {x}"
        state = {x: ref[x] for x in ("mate_a", "mate_b", "y_a", "y_b")}


def test_warm_start_rejects_bad_state(ctx):
    import paper_2203_03732_amd as prot
    n = 16
    k = synth.random_k(n, 4, seed=1)
    bad = dict(mate_a=np.full(n, -1, np.int32), mate_b=np.full(n, -1, np.int32),
               y_a=np.zeros(n, np.int32), y_b=np.ones(n, np.int32))
    bad["y_a"][3] = -1  # a free column with a nonzero dual violates (I1)
    with pytest.raises(prot.ProtError) as e:
        ctx.solve_rounded(padded_k(k), 0, n, state={x: dev(v) for x, v in bad.items()})
    assert e.value.name == "state"


def test_max_phases_partial(ctx):
    n, K, T = 300, 20, 3
    k = synth.random_k(n, K, seed=3)
    ref = oracle.solve_rounded(k, T, max_phases=2, complete=False)
    gpu = ctx.solve_rounded(padded_k(k), T, n, max_phases=2, complete=False)
    assert ref["status"] == "partial" and gpu.status == "partial"
    assert_same(gpu, ref)


def test_empty(ctx):
    gpu = ctx.solve_rounded(torch.empty((0, 128), dtype=torch.int16, device="cuda"), 0, 0)
    assert gpu.status == "ok" and gpu.stats["phases"] == 0


def test_deterministic(ctx):
    k = synth.random_k(2000, 40, seed=11)
    kd = padded_k(k)
    r1 = ctx.solve_rounded(kd, 20, 2000)
    r2 = ctx.solve_rounded(kd, 20, 2000)
    for x in ("mate_a", "mate_b", "y_a", "y_b"):
        assert torch.equal(getattr(r1, x), getattr(r2, x))
    for s in STAT_KEYS:
        assert r1.stats[s] == r2.stats[s]


# --------------------------------------------------- end to end workloads

def test_uniform_costs_n1000_eps01(ctx):
    """Uniform [0,1) costs, n = 1000, eps = 0.1."""
    n, eps = 1000, 0.1
    C = synth.uniform_costs(n, seed=0)
    gpu = ctx.solve_cost(dev(C), eps)
    k = oracle.round_cost(C, eps)
    orc = oracle.solve_rounded(k, oracle.threshold(eps, n), trace=True)
    assert_same(gpu, orc)
    cost = float(C.astype(np.float64)[np.arange(n), orc["mate_b"]].sum())
    assert math.isclose(gpu.stats["cost"], cost, rel_tol=1e-12)
    assert gpu.stats["threshold"] == 100


@pytest.mark.parametrize("eps_mode", ["algorithmic", "strict"])
def test_solve_cost_modes(ctx, eps_mode):
    n, eps = 400, 0.05
    C = synth.uniform_costs(n, seed=9)
    gpu = ctx.solve_cost(dev(C), eps, eps_mode=eps_mode)
    ei = eps / 3 if eps_mode == "strict" else eps
    orc = oracle.solve_rounded(oracle.round_cost(C, ei), oracle.threshold(ei, n))
    assert_same(gpu, orc)
    assert gpu.stats["eps_internal"] == ei


def _points_case(ctx, n, d, eps, seed=0, storage="matrix", origin="diag", X=None, Y=None):
    if X is None:
        X, Y = synth.uniform_points(n, d, seed=seed)
    gpu = ctx.solve_points(dev(X), dev(Y), eps, storage=storage, origin=origin)
    k, m = oracle.round_points_f32(X, Y, eps)
    orc = oracle.solve_rounded(k, oracle.threshold(eps, n), trace=True, origin=origin)
    assert_same(gpu, orc, f"points n={n} {storage} {origin}")
    for key in ("phases", "rounds", "scanned", "sum_free", "sum_k"):
        assert gpu.stats[key] == orc["stats"][key], key
    assert gpu.stats["cost_scale"] == m
    d2 = ((X.astype(np.float64) - Y.astype(np.float64)[orc["mate_b"]]) ** 2).sum(1)
    want = d2.sum() / m if m > 0 else 0.0  # all points equal: every cost is 0
    assert math.isclose(gpu.stats["cost"], want, rel_tol=1e-12, abs_tol=1e-300)
    return gpu, orc, k


@pytest.mark.parametrize("storage", ["matrix", "on_the_fly"])
def test_points_small(ctx, storage):
    _points_case(ctx, 2000, 2, 0.01, seed=4, storage=storage)
    _points_case(ctx, 1500, 3, 0.005, seed=5, storage=storage)


@pytest.mark.parametrize("origin", ["diag", "zero"])
@pytest.mark.parametrize("n,d,eps", [(1, 2, 0.1), (7, 3, 0.2), (13, 2, 0.05), (1001, 3, 0.01),
                                     (4099, 2, 0.02)])
def test_points_on_the_fly_ragged(ctx, n, d, eps, origin):
    """Costs recomputed in the greedy step: sizes that leave partial chunks,
    both scan origins; bit-exact with the matrix-free definition."""
    _points_case(ctx, n, d, eps, seed=n + d, storage="on_the_fly", origin=origin)


def test_points_on_the_fly_degenerate(ctx):
    """All points equal (m = 0, every k = 0) and clustered duplicates."""
    n = 300
    X = np.full((n, 2), 0.25, np.float32)
    _points_case(ctx, n, 2, 0.05, storage="on_the_fly", X=X, Y=X.copy())
    rng = np.random.default_rng(5)
    X = np.repeat(rng.random((30, 3), dtype=np.float32), 10, axis=0)
    Y = np.repeat(rng.random((30, 3), dtype=np.float32), 10, axis=0)
    _points_case(ctx, n, 3, 0.02, storage="on_the_fly", X=X, Y=Y)


def test_points_on_the_fly_rejects_high_d(ctx):
    import paper_2203_03732_amd as prot
    X, Y = synth.uniform_points(64, 5, seed=1)
    with pytest.raises(prot.ProtError) as e:
        ctx.solve_points(dev(X), dev(Y), 0.1, storage="on_the_fly")
    assert e.value.name == "unsupported"


@pytest.mark.parametrize("storage", ["matrix", "on_the_fly"])
def test_points_n10000_eps001(ctx, storage):
    """Two sets of 10k uniform points in the unit square, squared Euclidean
    cost scaled to max 1, eps = 0.01: bit-exact with the oracle end to end."""
    gpu, orc, k = _points_case(ctx, 10000, 2, 0.01, seed=0, storage=storage)
    assert np.array_equal(ctx.trace(), orc["trace"])


@pytest.fixture(scope="module")
def c5_oracle():
    """The oracle on the 3-D instance at full size (n = 50,000, eps =
    0.005), every examined cost computed from the points (no matrix)."""
    X, Y = synth.uniform_points(50000, 3, seed=0)
    return X, Y, oracle.solve_points(X, Y, 0.005, trace=True)


@pytest.mark.parametrize("storage", ["matrix", "on_the_fly"])
def test_points_n50000_d3_bit_exact(ctx, c5_oracle, storage):
    """n = 50,000 points in the unit cube, eps = 0.005, as the benchmark
    runs it: the 5 GB int16 matrix resident in HBM, and costs recomputed in
    the scan. Mates, duals, every statistic and the per-phase trace equal
    the oracle's, element by element."""
    X, Y, orc = c5_oracle
    gpu = ctx.solve_points(dev(X), dev(Y), 0.005, storage=storage)
    assert_same(gpu, orc, f"n=50000 {storage}")
    assert gpu.stats["cost_scale"] == orc["m"]
    assert np.array_equal(ctx.trace(), orc["trace"])


def test_points_n50000_d3_full_size_on_the_fly(ctx):
    """The 3-D instance at full size (n = 50,000, eps = 0.005) as the default
    runs it (costs on the fly): the maximum and every matched pair's rounded
    cost from the oracle, (I1), eq. (3) on the matching, (I2) on sampled full
    rows, Sigma k, and the dual certificate c(M) <= eps (Sigma y - n) + 3 eps n
    (c(OPT) >= eps (Sigma y - n) by eq. (2)); the matrix storage gives the
    identical result."""
    n, d, eps = 50000, 3, 0.005
    X, Y = synth.uniform_points(n, d, seed=0)
    Xd, Yd = dev(X), dev(Y)
    loop = ctx.solve_points(Xd, Yd, eps, complete=False)
    full = ctx.solve_points(Xd, Yd, eps)
    m = oracle.points_max_f32(X, Y)
    assert loop.stats["cost_scale"] == m and full.stats["cost_scale"] == m
    mate_a, mate_b = host(loop.mate_a), host(loop.mate_b)
    ya, yb = host(loop.y_a).astype(np.int64), host(loop.y_b).astype(np.int64)
    matched = np.nonzero(mate_b >= 0)[0]
    assert np.array_equal(mate_a[mate_b[matched]], matched)
    assert n - len(matched) <= oracle.threshold(eps, n)
    assert (yb >= 0).all() and (ya <= 0).all() and (ya[mate_a < 0] == 0).all()
    kp = oracle.points_pairs_f32(X, Y, eps, m, matched, mate_b[matched]).astype(np.int64)
    assert np.array_equal(ya[mate_b[matched]] + yb[matched], kp)  # eq. (3) on M
    assert loop.stats["sum_k"] == kp.sum()
    rng = np.random.default_rng(1)
    cols = np.arange(n)
    for b in rng.choice(n, 12, replace=False):
        kr = oracle.points_pairs_f32(X, Y, eps, m, np.full(n, b), cols).astype(np.int64)
        assert (ya + yb[b] <= kr + 1).all(), f"(I2) fails on row {b}"  # eq. (2)
    for x in ("y_a", "y_b"):
        assert torch.equal(getattr(loop, x), getattr(full, x))
    lb = eps * (ya.sum() + yb.sum() - n)
    assert full.stats["cost"] <= lb + 3 * eps * n + 1e-9
    same = ctx.solve_points(Xd, Yd, eps, storage="matrix")
    for x in ("mate_a", "mate_b", "y_a", "y_b"):
        assert torch.equal(getattr(same, x), getattr(full, x))
    for key in ("phases", "rounds", "scanned", "sum_k"):
        assert same.stats[key] == full.stats[key]


@pytest.fixture(scope="module")
def prune_ctx():
    """A context that prunes the maximum pass at every size (the default
    starts at n = 16384)."""
    import os
    import paper_2203_03732_amd as prot
    old = os.environ.get("PROT_PRUNE_MIN_N")
    os.environ["PROT_PRUNE_MIN_N"] = "0"
    try:
        c = prot.Context(0)
    finally:
        if old is None:
            del os.environ["PROT_PRUNE_MIN_N"]
        else:
            os.environ["PROT_PRUNE_MIN_N"] = old
    yield c
    torch.cuda.synchronize()
    c.close()


def _pruning_points(case, d):
    rng = np.random.default_rng(sum(map(ord, case)) + d)
    n = 1 if case == "one" else 700
    if case == "clusters":  # every cross pair is near the maximum: nothing pruned
        X = (rng.random((n, d)) * 1e-3).astype(np.float32)
        Y = (5.0 + rng.random((n, d)) * 1e-3).astype(np.float32)
    elif case == "equal":
        X = np.full((n, d), -3.5, np.float32)
        Y = X.copy()
    elif case == "negative":
        X = (-rng.random((n, d)) * 7).astype(np.float32)
        Y = (-rng.random((n, d)) * 3 - 2).astype(np.float32)
    elif case == "offset":
        X = (1000.0 + rng.standard_normal((n, d))).astype(np.float32)
        Y = (1000.0 + rng.standard_normal((n, d))).astype(np.float32)
    elif case == "line":
        t = rng.random(n).astype(np.float32)
        X = np.stack([t, 2 * t] + [t] * (d - 2), 1).astype(np.float32)
        Y = np.stack([1 - t, 2 - 2 * t] + [t] * (d - 2), 1).astype(np.float32)
    elif case == "sphere":
        v = rng.standard_normal((n, d))
        X = (v / np.linalg.norm(v, axis=1, keepdims=True)).astype(np.float32)
        w = rng.standard_normal((n, d))
        Y = (w / np.linalg.norm(w, axis=1, keepdims=True)).astype(np.float32)
    else:  # one point each
        X = rng.random((n, d), dtype=np.float32)
        Y = rng.random((n, d), dtype=np.float32)
    return np.ascontiguousarray(X), np.ascontiguousarray(Y)


@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("case", ["clusters", "equal", "one", "negative", "offset", "line",
                                  "sphere"])
def test_points_maximum_pruning_cases(prune_ctx, case, d):
    """The maximum over all pairs is found by pruning to candidate pairs; it
    must equal the definition's maximum bit for bit, in the cost build and in
    the solve with costs on the fly."""
    ctx = prune_ctx
    X, Y = _pruning_points(case, d)
    k, m = ctx.build_costs(dev(X), dev(Y), 0.05)
    torch.cuda.synchronize()
    ko, mo = oracle.round_points_f32(X, Y, 0.05)
    assert float(host(m)[0]) == mo
    assert np.array_equal(host(k)[:, :X.shape[0]], ko)
    gpu = ctx.solve_points(dev(X), dev(Y), 0.05, storage="on_the_fly")
    assert gpu.stats["cost_scale"] == mo


def test_max_phases_partial_leaves_state_uncompleted(ctx):
    """A loop stopped by max_phases is not completed even when completion is
    asked for: the state stays resumable, as the oracle leaves it."""
    n, K, T = 300, 20, 3
    k = synth.random_k(n, K, seed=13)
    ref = oracle.solve_rounded(k, T, max_phases=2)
    gpu = ctx.solve_rounded(padded_k(k), T, n, max_phases=2)
    assert ref["status"] == "partial" and gpu.status == "partial"
    assert ref["stats"]["completed_pairs"] == 0
    assert_same(gpu, ref)


@pytest.mark.parametrize("k_type", ["int16", "uint8"])
def test_matrix_element_types(ctx, k_type):
    """The stored matrix as int16 or as bytes (floor(1/eps) <= 253): the
    same results, on point sets (square and rectangular, both origins), on a
    cost matrix, and with the Euclidean cost."""
    for n, n_a, d, eps, origin in [(2000, 2000, 2, 0.01, "diag"), (1500, 2300, 3, 0.005, "zero"),
                                   (777, 777, 16, 0.05, "diag")]:
        X, Y = synth.uniform_points(n, d, seed=n + d, n_a=n_a)
        gpu = ctx.solve_points(dev(X), dev(Y), eps, origin=origin, storage="matrix",
                               k_type=k_type)
        k, _ = oracle.round_points_f32(X, Y, eps)
        orc = oracle.solve_rounded(k, oracle.threshold(eps, n), origin=origin)
        assert_same(gpu, orc, f"points {n}x{n_a} {k_type}")
    C = synth.uniform_costs(1000, seed=4)
    gpu = ctx.solve_cost(dev(C), 0.1, k_type=k_type)
    orc = oracle.solve_rounded(oracle.round_cost(C, 0.1), oracle.threshold(0.1, 1000))
    assert_same(gpu, orc, f"costs {k_type}")
    X, Y = synth.uniform_points(1200, 2, seed=8)
    ctx.set_cost_metric("euclidean")
    try:
        gpu = ctx.solve_points(dev(X), dev(Y), 0.01, k_type=k_type)
    finally:
        ctx.set_cost_metric("sqeuclidean")
    k, _ = oracle.round_points_euclid_f32(X, Y, 0.01)
    assert_same(gpu, oracle.solve_rounded(k, oracle.threshold(0.01, 1200)), f"euclid {k_type}")


def test_byte_matrix_needs_small_k(ctx):
    import paper_2203_03732_amd as prot
    X, Y = synth.uniform_points(300, 2, seed=2)
    with pytest.raises(prot.ProtError) as e:
        ctx.solve_points(dev(X), dev(Y), 0.002, k_type="uint8")  # floor(1/eps) = 500
    assert e.value.name == "unsupported"
    # the automatic choice keeps int16 there
    gpu = ctx.solve_points(dev(X), dev(Y), 0.002)
    k, _ = oracle.round_points_f32(X, Y, 0.002)
    assert_same(gpu, oracle.solve_rounded(k, oracle.threshold(0.002, 300)), "auto K=500")


@pytest.fixture(scope="module")
def gate_ctx():
    """A context whose phase-loop gate admits only three workgroups, as when
    the rest of the grid is not resident (the plain launch's partial case)."""
    import os
    import paper_2203_03732_amd as prot
    old = os.environ.get("PROT_LOOP_GATE_CAP")
    os.environ["PROT_LOOP_GATE_CAP"] = "3"
    try:
        c = prot.Context(0)
    finally:
        if old is None:
            del os.environ["PROT_LOOP_GATE_CAP"]
        else:
            os.environ["PROT_LOOP_GATE_CAP"] = old
    yield c
    torch.cuda.synchronize()
    c.close()


@pytest.mark.parametrize("n,eps,origin", [(1000, 0.01, "diag"), (2900, 0.02, "zero"), (64, 0.1, "diag")])
def test_loop_with_few_workgroups_admitted(gate_ctx, n, eps, origin):
    """Three workgroups (48 waves) serve every row: the result is the
    oracle's, bit for bit, as with the whole grid."""
    X, Y = synth.uniform_points(n, 2, seed=n)
    gpu = gate_ctx.solve_points(dev(X), dev(Y), eps, origin=origin)
    k, _ = oracle.round_points_f32(X, Y, eps)
    orc = oracle.solve_rounded(k, oracle.threshold(eps, n), origin=origin)
    for x in ("mate_a", "mate_b", "y_a", "y_b"):
        assert np.array_equal(host(getattr(gpu, x)), orc[x]), x
    for s in STAT_KEYS:
        assert gpu.stats[s] == orc["stats"][s], s


def test_loop_falls_back_to_a_cooperative_launch(gate_ctx):
    """3 workgroups x 16 waves x 64 lanes = 3,072 rows at most: with more rows
    the gated launch runs nothing (too few workgroups admitted) and the call
    runs the loop again with a cooperative launch, bit-exact with the oracle.
    Enqueued without statistics (no synchronisation, no retry) the failure
    is reported by the status query, and the outputs are marked invalid."""
    X, Y = synth.uniform_points(4000, 2, seed=2)
    gpu = gate_ctx.solve_points(dev(X), dev(Y), 0.05)
    k, _ = oracle.round_points_f32(X, Y, 0.05)
    orc = oracle.solve_rounded(k, oracle.threshold(0.05, 4000), trace=True)
    assert_same(gpu, orc, "cooperative fallback")
    import paper_2203_03732_amd as prot
    kd = padded_k(k)
    res = gate_ctx.solve_rounded(kd, oracle.threshold(0.05, 4000), 4000, stats=False)
    with pytest.raises(prot.ProtError) as e:
        gate_ctx.status()
    assert e.value.name == "hip"
    assert (host(res.mate_b) == -1).all()
    X, Y = synth.uniform_points(500, 2, seed=3)
    gpu = gate_ctx.solve_points(dev(X), dev(Y), 0.05)
    k, _ = oracle.round_points_f32(X, Y, 0.05)
    orc = oracle.solve_rounded(k, oracle.threshold(0.05, 500))
    assert np.array_equal(host(gpu.mate_b), orc["mate_b"])


# ------------------------------------------------ failing closed, watchdog
@pytest.mark.parametrize("origin", ["diag", "zero"])
def test_watchdog_stops_with_the_state_of_that_many_phases(ctx, origin):
    """phase_bound = 3: the call stops after three phases with status
    phase_bound (no completion) and the state equals the oracle's after
    three phases; resuming it (default watchdog) finishes like one run."""
    n, eps = 3000, 0.01
    X, Y = synth.uniform_points(n, 2, seed=21)
    k, _ = oracle.round_points_f32(X, Y, eps)
    T = oracle.threshold(eps, n)
    kd = padded_k(k)
    part = ctx.solve_rounded(kd, T, n, origin=origin, phase_bound=3)
    assert part.status == "phase_bound"
    ref = oracle.solve_rounded(k, T, origin=origin, max_phases=3, complete=False)
    assert_same(part, ref, "watchdog at 3 phases")
    rest = ctx.solve_rounded(kd, T, n, origin=origin, state=dict(
        mate_a=part.mate_a, mate_b=part.mate_b, y_a=part.y_a, y_b=part.y_b), check_warm=True)
    full = oracle.solve_rounded(k, T, origin=origin)
    for x in ("mate_a", "mate_b", "y_a", "y_b"):
        assert np.array_equal(host(getattr(rest, x)), full[x]), x
    assert part.stats["phases"] + rest.stats["phases"] == full["stats"]["phases"]
    # the same stop through the asynchronous path and the status query
    again = ctx.solve_rounded(kd, T, n, origin=origin, phase_bound=3, stats=False)
    assert ctx.status() == "phase_bound"
    for x in ("mate_a", "mate_b", "y_a", "y_b"):
        assert torch.equal(getattr(again, x), getattr(part, x)), x


def test_points_watchdog(ctx):
    """The watchdog on a point-set solve (costs on the fly) stops at the
    given phase count with the oracle's state."""
    n, eps = 2000, 0.02
    X, Y = synth.uniform_points(n, 3, seed=22)
    gpu = ctx.solve_points(dev(X), dev(Y), eps, storage="on_the_fly", phase_bound=2)
    assert gpu.status == "phase_bound" and gpu.stats["phases"] == 2
    ref = oracle.solve_points(X, Y, eps, max_phases=2, complete=False)
    assert_same(gpu, ref, "points watchdog")


def test_warm_start_checks(ctx):
    """Warm starts: (I2) checked on request (a state from the oracle passes;
    one dual raised by one step fails it); a dual beyond Lemma 3.2's range
    is refused; a free row whose dual would leave its 15-bit field stops the
    loop with an error and the outputs marked invalid."""
    import paper_2203_03732_amd as prot
    n, eps = 800, 0.05
    X, Y = synth.uniform_points(n, 2, seed=23)
    k, _ = oracle.round_points_f32(X, Y, eps)
    T = oracle.threshold(eps, n)
    kd = padded_k(k)
    ref = oracle.solve_rounded(k, T, max_phases=2, complete=False)
    st = {x: dev(ref[x]) for x in ("mate_a", "mate_b", "y_a", "y_b")}
    ok = ctx.solve_rounded(kd, T, n, state=st, check_warm=True)
    full = oracle.solve_rounded(k, T)
    assert np.array_equal(host(ok.mate_b), full["mate_b"])
    bad = dict(st)
    yb = ref["y_b"].copy()
    b = int(np.nonzero(ref["mate_b"] >= 0)[0][0])
    yb[b] += 1  # eq. (3) fails on b's matched edge
    bad["y_b"] = dev(yb)
    with pytest.raises(prot.ProtError) as e:
        ctx.solve_rounded(kd, T, n, state=bad, check_warm=True)
    assert e.value.name == "state"
    yb = ref["y_b"].copy()
    yb[b] = 40000  # beyond |y| <= K + 2 for any int16 matrix
    bad["y_b"] = dev(yb)
    with pytest.raises(prot.ProtError) as e:
        ctx.solve_rounded(kd, T, n, state=bad)
    assert e.value.name == "state"
    # all-zero costs, one free row with y(b) = 32767: it finds no column
    # (it would need k = 32766) and its dual cannot grow
    m = 64
    z = np.zeros((m, m), np.int16)
    mate = np.arange(m, dtype=np.int32)
    mate_a, mate_b = mate.copy(), mate.copy()
    mate_a[5] = -1
    mate_b[5] = -1
    y_a = np.zeros(m, np.int32)
    y_b = np.zeros(m, np.int32)
    y_b[5] = 32767
    over = dict(mate_a=dev(mate_a), mate_b=dev(mate_b), y_a=dev(y_a), y_b=dev(y_b))
    with pytest.raises(prot.ProtError) as e:
        ctx.solve_rounded(padded_k(z), 0, m, state=over)
    assert e.value.name == "state" and "Lemma 3.2" in str(e.value)
    # the context still solves afterwards
    gpu = ctx.solve_rounded(kd, T, n)
    assert_same(gpu, full, "after the failures")


def test_barrier_timeout_fails_closed():
    """A context whose round-barrier wait is cut to ~10 ns: workgroups give
    up at the first barrier that is not already complete, every one of them
    leaves the loop (each wait is bounded), the call reports the time-out
    and marks the outputs invalid; a normal context then solves."""
    import os
    import paper_2203_03732_amd as prot
    old = os.environ.get("PROT_LOOP_BARRIER_TICKS")
    os.environ["PROT_LOOP_BARRIER_TICKS"] = "1"
    try:
        c = prot.Context(0)
    finally:
        if old is None:
            del os.environ["PROT_LOOP_BARRIER_TICKS"]
        else:
            os.environ["PROT_LOOP_BARRIER_TICKS"] = old
    n, eps = 6000, 0.01
    X, Y = synth.uniform_points(n, 2, seed=24)
    k, _ = oracle.round_points_f32(X, Y, eps)
    kd = padded_k(k)
    try:
        res = c.solve_rounded(kd, oracle.threshold(eps, n), n, stats=False)
        with pytest.raises(prot.ProtError) as e:
            c.status()
        assert e.value.name == "hip" and "barrier" in str(e.value)
        assert (host(res.mate_b) == -1).all() and (host(res.mate_a) == -1).all()
    finally:
        torch.cuda.synchronize()
        c.close()
    c2 = prot.Context(0)
    gpu = c2.solve_rounded(kd, oracle.threshold(eps, n), n)
    assert_same(gpu, oracle.solve_rounded(k, oracle.threshold(eps, n)), "after the time-out")
    c2.close()
