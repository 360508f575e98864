"""GPU parity for the unbalanced case (Section 3.3, Lemma 3.5): n_b rows
(supply B) and n_a >= n_b columns (demand A), through the rectangular C
calls, against the CPU oracle on the same inputs. Matchings, duals,
statistics and the per-phase trace must be bit-exact; rounded costs are
bit-exact with the oracle's definitions."""
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
    """Device copy of an n_b x n_a int16 matrix in the pitched layout, padded
    with the largest int16 so a read past n_a would show."""
    import paper_2203_03732_amd as prot
    n_b, n_a = k_np.shape
    kp = np.full((n_b, prot.pitch(n_a)), 0x7FFF, np.int16)
    kp[:, :n_a] = k_np
    return dev(kp)


def assert_same(gpu, orc, what=""):
    for x in ("mate_a", "mate_b", "y_a", "y_b"):
        g = host(getattr(gpu, x))
        assert g.shape == orc[x].shape, f"{what}: {x} shape {g.shape} != {orc[x].shape}"
        assert np.array_equal(g, orc[x]), f"{what}: {x} differs at {np.nonzero(g != orc[x])[0][:10]}"
    for s in STAT_KEYS:
        assert gpu.stats[s] == orc["stats"][s], f"{what}: stat {s} {gpu.stats[s]} != {orc['stats'][s]}"


RECT = [(1, 5, 3, 0), (3, 700, 9, 0), (37, 100, 9, 1), (300, 301, 20, 3), (500, 1500, 15, 5),
        (1000, 4100, 30, 10), (1024, 1025, 7, 0), (2000, 2999, 40, 20), (64, 20000, 12, 0)]


@pytest.mark.parametrize("origin", ["diag", "zero"])
@pytest.mark.parametrize("n_b,n_a,K,T", RECT)
def test_solve_rounded_rect_bit_exact(ctx, n_b, n_a, K, T, origin):
    k = synth.random_k(n_b, K, seed=n_b * 7 + n_a, n_a=n_a)
    orc = oracle.solve_rounded(k, T, origin=origin, trace=True)
    gpu = ctx.solve_rounded(padded_k(k), T, n_b, n_a=n_a, origin=origin)
    assert gpu.status == "ok"
    assert_same(gpu, orc, f"n_b={n_b} n_a={n_a} K={K} T={T} {origin}")
    assert np.array_equal(ctx.trace(), orc["trace"])
    mate_a = host(gpu.mate_a)
    check_matching(mate_a, host(gpu.mate_b), perfect=True)
    assert int((mate_a < 0).sum()) == n_a - n_b


def test_single_row_closed_form(ctx):
    """One row over five columns: the phases raise y(b) until the cheapest
    column (first of the two with k = 3) is admissible."""
    k = np.array([[5, 3, 7, 3, 9]], np.int16)
    gpu = ctx.solve_rounded(padded_k(k), 0, 1, n_a=5)
    assert gpu.stats["phases"] == 4
    assert host(gpu.mate_b).tolist() == [1]
    assert host(gpu.y_b).tolist() == [4]
    assert host(gpu.y_a).tolist() == [0, -1, 0, 0, 0]
    assert host(gpu.mate_a).tolist() == [-1, 0, -1, -1, -1]


@pytest.mark.parametrize("origin", ["diag", "zero"])
def test_rect_structured(ctx, origin):
    n_b, n_a = 200, 333
    r, c = np.arange(n_b)[:, None], np.arange(n_a)[None, :]
    cases = {"zeros": np.zeros((n_b, n_a), np.int16),
             "band": np.where(np.abs(r - c) < 2, 0, 9).astype(np.int16),
             "ramp": ((r + c) % 13).astype(np.int16),
             "rows": np.repeat((np.arange(n_b) % 5)[:, None], n_a, 1).astype(np.int16),
             "cols": np.repeat((np.arange(n_a) % 5)[None, :], n_b, 0).astype(np.int16),
             "late": np.repeat(np.where(c >= n_a - n_b, 0, 20), n_b, 0).astype(np.int16)}
    for name, k in cases.items():
        assert k.shape == (n_b, n_a), name
        orc = oracle.solve_rounded(k, 2, origin=origin)
        gpu = ctx.solve_rounded(padded_k(k), 2, n_b, n_a=n_a, origin=origin)
        assert_same(gpu, orc, name)


def test_rect_no_completion_invariants(ctx):
    n_b, n_a, K, T = 400, 900, 25, 12
    k = synth.random_k(n_b, K, seed=5, n_a=n_a)
    orc = oracle.solve_rounded(k, T, complete=False)
    gpu = ctx.solve_rounded(padded_k(k), T, n_b, n_a=n_a, complete=False)
    assert_same(gpu, orc)
    check_matching(host(gpu.mate_a), host(gpu.mate_b))
    check_I1(host(gpu.mate_a), host(gpu.y_a), host(gpu.y_b))
    check_I2(k, host(gpu.mate_b), host(gpu.y_a), host(gpu.y_b))
    assert int((host(gpu.mate_b) < 0).sum()) <= T


def test_rect_warm_start_and_max_phases(ctx):
    """Resume on the GPU from the oracle's state after p phases, one phase
    at a time, on a rectangular instance."""
    n_b, n_a, K, T = 300, 330, 60, 2
    k = synth.random_k(n_b, K, seed=19, n_a=n_a)
    kd = padded_k(k)
    full = oracle.solve_rounded(k, T, complete=False)
    assert full["stats"]["phases"] > 3
    state = None
    for p in range(full["stats"]["phases"]):
        ref = oracle.solve_rounded(k, T, max_phases=1, state=state, complete=False)
        st_dev = None if state is None else {x: dev(state[x]) for x in state}
        gpu = ctx.solve_rounded(kd, T, n_b, n_a=n_a, state=st_dev, max_phases=1,
                                complete=False)
        for x in ("mate_a", "mate_b", "y_a", "y_b"):
            assert np.array_equal(host(getattr(gpu, x)), ref[x]), f"phase {p}: {x}"
        state = {x: ref[x] for x in ("mate_a", "mate_b", "y_a", "y_b")}
    ref = oracle.solve_rounded(k, T, max_phases=2, complete=False)
    gpu = ctx.solve_rounded(kd, T, n_b, n_a=n_a, max_phases=2, complete=False)
    assert ref["status"] == "partial" and gpu.status == "partial"
    assert_same(gpu, ref)


def test_rect_rejects_more_rows_than_columns(ctx):
    import paper_2203_03732_amd as prot
    k = synth.random_k(10, 4, seed=1, n_a=10)
    with pytest.raises(prot.ProtError) as e:
        ctx.solve_rounded(padded_k(k), 0, 10, n_a=9)
    assert e.value.name == "arg"
    C = synth.uniform_costs(12, seed=1, n_a=8)
    with pytest.raises(prot.ProtError) as e:
        ctx.solve_cost(dev(C), 0.1)
    assert e.value.name == "arg"
    X, Y = synth.uniform_points(12, 2, seed=1, n_a=8)
    with pytest.raises(prot.ProtError) as e:
        ctx.solve_points(dev(X), dev(Y), 0.1)
    assert e.value.name == "arg"


def test_rect_no_rows(ctx):
    gpu = ctx.solve_rounded(torch.empty((0, 16), dtype=torch.int16, device="cuda"), 0, 0,
                            n_a=13)
    assert gpu.status == "ok" and gpu.stats["phases"] == 0
    assert host(gpu.mate_a).tolist() == [-1] * 13
    assert host(gpu.y_a).tolist() == [0] * 13
    X, Y = synth.uniform_points(0, 2, seed=0, n_a=9)
    gpu = ctx.solve_points(dev(X), dev(Y), 0.1)
    assert host(gpu.mate_a).tolist() == [-1] * 9 and gpu.mate_b.numel() == 0


@pytest.mark.parametrize("n_b,n_a,eps", [(1, 3, 0.1), (37, 41, 0.1), (300, 1000, 0.01),
                                         (777, 1111, 0.003)])
def test_round_costs_rect_bit_exact(ctx, n_b, n_a, eps):
    C = synth.uniform_costs(n_b, seed=n_b + n_a, n_a=n_a)
    k = ctx.round_costs(dev(C), eps)
    torch.cuda.synchronize()
    assert np.array_equal(host(k)[:, :n_a], oracle.round_cost(C, eps))


@pytest.mark.parametrize("path", ["direct", "matrix_cores"])
@pytest.mark.parametrize("n_b,n_a,d,eps", [(1, 9, 2, 0.1), (50, 77, 3, 0.01),
                                           (1000, 2500, 2, 0.01), (333, 1500, 16, 0.02)])
def test_build_costs_rect_bit_exact(ctx, n_b, n_a, d, eps, path):
    X, Y = synth.uniform_points(n_b, d, seed=n_a, n_a=n_a)
    ctx.set_cost_path(path)
    try:
        k, m = ctx.build_costs(dev(X), dev(Y), eps)
        torch.cuda.synchronize()
    finally:
        ctx.set_cost_path("auto")
    ko, mo = oracle.round_points_f32(X, Y, eps)
    assert float(host(m)[0]) == mo
    assert np.array_equal(host(k)[:, :n_a], ko)


@pytest.mark.parametrize("eps_mode", ["algorithmic", "strict"])
def test_solve_cost_rect(ctx, eps_mode):
    n_b, n_a, eps = 400, 1000, 0.05
    C = synth.uniform_costs(n_b, seed=9, n_a=n_a)
    gpu = ctx.solve_cost(dev(C), eps, eps_mode=eps_mode)
    ei = eps / 3 if eps_mode == "strict" else eps
    T = oracle.threshold(ei, n_b)
    assert gpu.stats["threshold"] == T
    orc = oracle.solve_rounded(oracle.round_cost(C, ei), T)
    assert_same(gpu, orc)
    cost = float(C.astype(np.float64)[np.arange(n_b), orc["mate_b"]].sum())
    assert math.isclose(gpu.stats["cost"], cost, rel_tol=1e-12)


def _points_rect(ctx, n_b, n_a, d, eps, seed, storage, origin="diag"):
    X, Y = synth.uniform_points(n_b, d, seed=seed, n_a=n_a)
    gpu = ctx.solve_points(dev(X), dev(Y), eps, storage=storage, origin=origin)
    k, m = oracle.round_points_f32(X, Y, eps)
    orc = oracle.solve_rounded(k, oracle.threshold(eps, n_b), trace=True, origin=origin)
    assert_same(gpu, orc, f"points {n_b}x{n_a} d={d} {storage} {origin}")
    assert np.array_equal(ctx.trace(), orc["trace"])
    assert gpu.stats["cost_scale"] == m
    d2 = ((X.astype(np.float64) - Y.astype(np.float64)[orc["mate_b"]]) ** 2).sum(1)
    assert math.isclose(gpu.stats["cost"], d2.sum() / m, rel_tol=1e-12)


@pytest.mark.parametrize("origin", ["diag", "zero"])
@pytest.mark.parametrize("storage", ["matrix", "on_the_fly"])
@pytest.mark.parametrize("n_b,n_a,d,eps", [(7, 13, 2, 0.2), (1001, 1500, 3, 0.01),
                                           (1500, 4099, 2, 0.02), (5000, 6000, 2, 0.01)])
def test_points_rect(ctx, n_b, n_a, d, eps, storage, origin):
    _points_rect(ctx, n_b, n_a, d, eps, n_b + n_a, storage, origin)


@pytest.fixture(scope="module")
def prune_ctx():
    """A context that prunes the maximum pass at every size."""
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


@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("n_b,n_a", [(1, 700), (300, 2000), (999, 1000)])
def test_points_rect_pruned_maximum(prune_ctx, n_b, n_a, d):
    """The pruned maximum pass over n_b x n_a pairs equals the definition's."""
    rng = np.random.default_rng(n_b * 3 + d)
    X = (rng.standard_normal((n_b, d)) * 2 + 1).astype(np.float32)
    Y = rng.random((n_a, d), dtype=np.float32)
    k, m = prune_ctx.build_costs(dev(X), dev(Y), 0.05)
    torch.cuda.synchronize()
    ko, mo = oracle.round_points_f32(X, Y, 0.05)
    assert float(host(m)[0]) == mo
    assert np.array_equal(host(k)[:, :n_a], ko)
    gpu = prune_ctx.solve_points(dev(X), dev(Y), 0.05, storage="on_the_fly")
    assert gpu.stats["cost_scale"] == mo
    orc = oracle.solve_rounded(ko, oracle.threshold(0.05, n_b))
    assert_same(gpu, orc, "pruned rect")


def test_points_rect_large_auto(ctx):
    """20,000 rows in [0, 0.5]^2 over 30,000 columns in the unit square,
    eps = 0.01, as the library chooses to run it (pruned maximum; costs on
    the fly once the matrix outgrows the cache), against the oracle on the
    full instance (164 phases: most rows must reach outside their square)."""
    n_b, n_a, eps = 20000, 30000, 0.01
    X, Y = synth.uniform_points(n_b, 2, seed=3, n_a=n_a)
    X = (X * 0.5).astype(np.float32)
    gpu = ctx.solve_points(dev(X), dev(Y), eps)
    k, m = oracle.round_points_f32(X, Y, eps)
    orc = oracle.solve_rounded(k, oracle.threshold(eps, n_b))
    del k
    assert orc["stats"]["phases"] > 100
    assert gpu.stats["cost_scale"] == m
    assert_same(gpu, orc, "20000x30000")


def test_rect_at_the_column_limit(ctx):
    """The column duals live in one workgroup's LDS (2 bytes each): 80,000
    columns is close to the limit and runs there; 90,000 go past it, and
    each workgroup keeps its copy of the duals in global memory."""
    n_b, n_a, K, T = 200, 80000, 10, 2
    k = (20 + synth.random_k(n_b, K, seed=41, n_a=n_a)).astype(np.int16)  # ~20 empty phases
    orc = oracle.solve_rounded(k, T)
    gpu = ctx.solve_rounded(padded_k(k), T, n_b, n_a=n_a)
    assert_same(gpu, orc, "80000 columns")
    X, Y = synth.uniform_points(300, 2, seed=42, n_a=80000)
    gpu = ctx.solve_points(dev(X), dev(Y), 0.01, storage="on_the_fly")
    kk, m = oracle.round_points_f32(X, Y, 0.01)
    assert_same(gpu, oracle.solve_rounded(kk, oracle.threshold(0.01, 300)), "80000 on the fly")
    X, Y = synth.uniform_points(10, 2, seed=43, n_a=90000)
    gpu = ctx.solve_points(dev(X), dev(Y), 0.1)
    kk, m = oracle.round_points_f32(X, Y, 0.1)
    assert_same(gpu, oracle.solve_rounded(kk, oracle.threshold(0.1, 10)), "90000 columns")
    k = (20 + synth.random_k(n_b, K, seed=44, n_a=90000)).astype(np.int16)
    gpu = ctx.solve_rounded(padded_k(k), T, n_b, n_a=90000)
    assert_same(gpu, oracle.solve_rounded(k, T), "90000 columns, matrix")
