"""GPU parity for transport with the copies kept as two dual clusters
(Section 4, Lemma 4.1): prot_ot_solve_clustered through the C ABI against
the oracle's orc_ot_solve_clustered on the same inputs. The plan and the
repaired mass must be bit-exact, the duals (smaller dual of each point's
copies and how many hold it) and the statistics equal, the per-phase record
equal; the plan's cost agrees to rounding order."""
import math
import os

import numpy as np
import pytest

import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

STAT_KEYS = ("phases", "sum_free", "rounds", "max_rounds", "scanned",
             "matched_in_phases", "completed_pairs", "sum_k", "threshold")


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


def _masses(rng, n, zeros=0):
    w = rng.random(n) + 0.05
    if zeros:
        w[rng.choice(n, zeros, replace=False)] = 0.0
    return w / w.sum()


def _instance(n_b, n_a, seed, zeros=0, points=False, shift=0.0):
    if points:
        from paper_2203_03732_amd import synth
        return synth.transport_clouds(n_b, n_a, seed=seed, shift=shift)
    rng = np.random.default_rng(seed)
    C = rng.random((n_b, n_a)).astype(np.float32)
    return C, _masses(rng, n_b, zeros), _masses(rng, n_a)


def _duals(orc):
    """(b_lo, b_nlo, a_lo, a_nlo) from the oracle's clusters."""
    s, d = orc["s"], orc["d"]
    b_lo = np.where(s == 0, 0, np.where(orc["b_lo"] > 0, orc["Y"] - 1, orc["Y"]))
    b_n = np.where(s == 0, 0, np.where(orc["b_lo"] > 0, orc["b_lo"], s))
    a_lo = np.where(d == 0, 0, np.where(orc["a_bot"] > 0, orc["Z"] - 1, orc["Z"]))
    a_n = np.where(d == 0, 0, np.where(orc["a_bot"] > 0, orc["a_bot"], d))
    return [np.asarray(x, np.int32) for x in (b_lo, b_n, a_lo, a_n)]


def _compare(ctx, gpu, orc, what, plan=True):
    st = gpu.stats
    assert st["theta"] == orc["theta"], what
    assert st["copies_b"] == int(orc["s"].sum()) and st["copies_a"] == int(orc["d"].sum()), what
    for k in STAT_KEYS:
        want = orc["T"] if k == "threshold" else orc["stats"][k]
        assert st[k] == want, f"{what}: stat {k} {st[k]} != {want}"
    want = _duals(orc)
    got = [host(x) for x in (gpu.y_b_lo, gpu.y_b_nlo, gpu.y_a_lo, gpu.y_a_nlo)]
    for name, g, w in zip(("b_lo", "b_nlo", "a_lo", "a_nlo"), got, want):
        assert np.array_equal(g, w), f"{what}: {name} differs at {np.argwhere(g != w)[:5].tolist()}"
    tr = ctx.trace()
    assert np.array_equal(tr, orc["trace"][:len(tr)]) and len(tr) == min(len(orc["trace"]), 65536), \
        f"{what}: per-phase record differs"
    if plan:
        P = host(gpu.plan)
        assert np.array_equal(P, orc["plan"]), \
            f"{what}: plan differs at {np.argwhere(P != orc['plan'])[:5].tolist()}"
        assert st["repaired_mass"] == orc["repaired"], what
        assert math.isclose(st["cost"], orc["cost"], rel_tol=1e-12, abs_tol=1e-15), what


def _run(ctx, C, nu, mu, eps, origin="diag", max_phases=0):
    print(f"clustered OT {C.shape} eps={eps} {origin} max_phases={max_phases}", flush=True)
    orc = oracle.ot_solve_clustered(C, nu, mu, eps, origin=origin, max_phases=max_phases,
                                    trace=True)
    gpu = ctx.ot_solve(dev(C), dev(nu), dev(mu), eps, origin=origin, max_phases=max_phases,
                       clustered=True)
    return gpu, orc


@pytest.mark.parametrize("origin", ["diag", "zero"])
@pytest.mark.parametrize("n_b,n_a,eps,seed,zeros", [
    (1, 1, 0.1, 0, 0), (5, 7, 0.1, 1, 0), (9, 4, 0.2, 2, 1), (40, 40, 0.05, 3, 3),
    (100, 150, 0.02, 4, 0), (257, 130, 0.05, 5, 7), (130, 257, 0.01, 8, 0),
    (300, 300, 0.02, 6, 0), (1025, 70, 0.05, 7, 0)])
def test_clustered_bit_exact(ctx, n_b, n_a, eps, seed, zeros, origin):
    C, nu, mu = _instance(n_b, n_a, seed, zeros)
    gpu, orc = _run(ctx, C, nu, mu, eps, origin)
    assert gpu.status == "ok" and orc["status"] == "ok"
    _compare(ctx, gpu, orc, f"{n_b}x{n_a} eps={eps} seed={seed} {origin}")


def test_clustered_clouds_eps_001_n1000(ctx):
    """Two 1,000-point clouds, the demand one shifted by 1, random masses,
    eps = 0.01: theta = 400,000, far past what explicit copies allow."""
    C, nu, mu = _instance(1000, 1000, 11, points=True, shift=1.0)
    gpu, orc = _run(ctx, C, nu, mu, 0.01)
    assert gpu.status == "ok"
    _compare(ctx, gpu, orc, "clouds eps=0.01")
    assert orc["stats"]["phases"] > 100


@pytest.mark.parametrize("phases", [1, 2, 7])
def test_clustered_partial_state(ctx, phases):
    """Stopped after a few phases: the duals hold the oracle's state then."""
    C, nu, mu = _instance(60, 80, 21, points=True, shift=0.5)
    gpu, orc = _run(ctx, C, nu, mu, 0.02, max_phases=phases)
    assert gpu.status == "partial" and orc["status"] == "partial"
    _compare(ctx, gpu, orc, f"partial {phases}", plan=False)


@pytest.mark.parametrize("value", [0.0, 0.5, 1.0])
def test_clustered_constant_costs(ctx, value):
    """Every edge of a phase is admissible for every supply point: the
    longest admissible lists (part of them outside LDS at n = 2000)."""
    rng = np.random.default_rng(3)
    for n_b, n_a in ((50, 60), (2000, 2000)):
        C = np.full((n_b, n_a), value, np.float32)
        nu, mu = _masses(rng, n_b), _masses(rng, n_a)
        gpu, orc = _run(ctx, C, nu, mu, 0.05)
        _compare(ctx, gpu, orc, f"constant {value} {n_b}x{n_a}")


def test_clustered_lists_outside_lds(ctx):
    """With the LDS list area capped at 64 entries most admissible lists go
    to the global overflow area; the results do not change."""
    C, nu, mu = _instance(300, 200, 31, points=True, shift=0.3)
    os.environ["PROT_CLUSTER_LIST_CAP"] = "64"
    try:
        gpu, orc = _run(ctx, C, nu, mu, 0.02)
    finally:
        del os.environ["PROT_CLUSTER_LIST_CAP"]
    _compare(ctx, gpu, orc, "lists outside LDS")


def test_clustered_largest_size(ctx):
    """4,096 points a side (the most one workgroup holds)."""
    C, nu, mu = _instance(4096, 4096, 41, points=True, shift=1.0)
    gpu, orc = _run(ctx, C, nu, mu, 0.1)
    _compare(ctx, gpu, orc, "4096 x 4096")


def test_clustered_rejections(ctx):
    import paper_2203_03732_amd as prot
    C, nu, mu = _instance(4097, 3, 1)
    with pytest.raises(prot.ProtError, match="unsupported"):
        ctx.ot_solve(dev(C), dev(nu), dev(mu), 0.1, clustered=True)
    C, nu, mu = _instance(5, 5, 2)
    with pytest.raises(prot.ProtError, match="range"):
        ctx.ot_solve(dev(C), dev(nu * 2), dev(mu), 0.1, clustered=True)
    C[1, 1] = 1.5
    with pytest.raises(prot.ProtError, match="range"):
        ctx.ot_solve(dev(C), dev(nu), dev(mu), 0.1, clustered=True)


@pytest.mark.parametrize("grid", ["1", "2", "3"])
def test_clustered_small_grids(ctx, grid):
    """Workgroup 0 alone lists the rows (grid 1), or one or two others do:
    the results do not depend on who lists them."""
    C, nu, mu = _instance(300, 280, 51, points=True, shift=0.4)
    os.environ["PROT_CLUSTER_GRID"] = grid
    try:
        gpu, orc = _run(ctx, C, nu, mu, 0.02)
    finally:
        del os.environ["PROT_CLUSTER_GRID"]
    _compare(ctx, gpu, orc, f"grid {grid}")
