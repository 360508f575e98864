"""Column duals beyond LDS and rows beyond 17 bits (Section 2.2 scan,
Lemma 3.4, at sizes past one workgroup's LDS).

With more columns than LDS holds, each workgroup keeps its copy of the
column duals in global memory; with more than 131,071 rows, rows travel in
18 bits of the keys and free lists. Both modes can be forced at any size
(PROT_LOOP_T_GLOBAL=1, PROT_LOOP_WIDE_ROWS=1), which makes them checkable
bit for bit against the oracle at sizes it finishes in seconds; the
150,000-point instance that needs them is checked by the dual certificate."""
import os

import numpy as np
import pytest

import oracle
from paper_2203_03732_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

STAT_KEYS = ("phases", "sum_free", "rounds", "max_rounds", "scanned",
             "matched_in_phases", "completed_pairs", "sum_k")


def _context(**env):
    import paper_2203_03732_amd as prot
    old = {k: os.environ.get(k) for k in env}
    os.environ.update(env)
    try:
        return prot.Context(0)
    finally:
        for k, v in old.items():
            if v is None:
                del os.environ[k]
            else:
                os.environ[k] = v


@pytest.fixture(scope="module")
def forced():
    """Column duals in global memory and 18-bit rows at every size."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = _context(PROT_LOOP_T_GLOBAL="1", PROT_LOOP_WIDE_ROWS="1")
    yield c
    torch.cuda.synchronize()
    c.close()


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = _context()
    yield c
    torch.cuda.synchronize()
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.cpu().numpy()


def assert_same(gpu, orc, what):
    for x in ("mate_a", "mate_b", "y_a", "y_b"):
        g = host(getattr(gpu, x))
        assert np.array_equal(g, orc[x]), f"{what}: {x} differs at {np.nonzero(g != orc[x])[0][:10]}"
    for s in STAT_KEYS:
        assert gpu.stats[s] == orc["stats"][s], f"{what}: stat {s} {gpu.stats[s]} != {orc['stats'][s]}"


def padded_k(k_np):
    import paper_2203_03732_amd as prot
    n_b, n_a = k_np.shape
    kp = np.full((n_b, prot.pitch(n_a)), 0x7FFF, np.int16)
    kp[:, :n_a] = k_np
    return dev(kp)


@pytest.mark.parametrize("origin", ["diag", "zero"])
@pytest.mark.parametrize("n,K,T,seed", [(1, 5, 0, 0), (9, 3, 0, 1), (200, 10, 2, 2),
                                        (1000, 20, 10, 3), (777, 300, 7, 4)])
def test_rounded_forced_modes_bit_exact(forced, n, K, T, seed, origin):
    print(f"forced modes: rounded n={n} K={K} T={T} {origin}", flush=True)
    rng = np.random.default_rng(seed)
    k = rng.integers(0, K + 1, (n, n)).astype(np.int16)
    orc = oracle.solve_rounded(k, T, origin, trace=True)
    gpu = forced.solve_rounded(padded_k(k), T, n, origin=origin)
    assert_same(gpu, orc, f"rounded n={n}")
    assert np.array_equal(forced.trace(), orc["trace"])


@pytest.mark.parametrize("origin", ["diag", "zero"])
def test_rectangular_forced_modes_bit_exact(forced, origin):
    rng = np.random.default_rng(5)
    k = rng.integers(0, 30, (300, 1100)).astype(np.int16)
    orc = oracle.solve_rounded(k, 3, origin)
    gpu = forced.solve_rounded(padded_k(k), 3, 300, n_a=1100, origin=origin)
    assert_same(gpu, orc, f"rect {origin}")


@pytest.mark.parametrize("n,d,eps,storage", [(3000, 2, 0.01, "on_the_fly"),
                                             (2500, 3, 0.02, "on_the_fly"),
                                             (2000, 2, 0.05, "matrix")])
def test_points_forced_modes_bit_exact(forced, n, d, eps, storage):
    print(f"forced modes: points n={n} d={d} eps={eps} {storage}", flush=True)
    X, Y = synth.uniform_points(n, d, seed=n + d)
    orc = oracle.solve_points(X, Y, eps, trace=True)
    gpu = forced.solve_points(dev(X), dev(Y), eps, storage=storage)
    assert_same(gpu, orc, f"points n={n} d={d}")
    assert np.array_equal(forced.trace(), orc["trace"])


def test_points_n10000_forced_modes_bit_exact(forced):
    """The 10,000-point plane instance of the benchmark, end to end."""
    X, Y = synth.uniform_points(10000, 2, seed=0)
    orc = oracle.solve_points(X, Y, 0.01, trace=True)
    for storage in ("matrix", "on_the_fly"):
        print(f"forced modes: n=10000 {storage}", flush=True)
        gpu = forced.solve_points(dev(X), dev(Y), 0.01, storage=storage)
        assert_same(gpu, orc, f"n=10000 {storage}")
        assert np.array_equal(forced.trace(), orc["trace"])


def test_warm_start_forced_modes(forced):
    """Phase by phase through warm starts equals one run."""
    rng = np.random.default_rng(11)
    n = 400
    k = rng.integers(0, 25, (n, n)).astype(np.int16)
    orc = oracle.solve_rounded(k, 4, "diag")
    kd = padded_k(k)
    state = None
    for _ in range(200):
        gpu = forced.solve_rounded(kd, 4, n, max_phases=1, state=state, complete=False)
        state = {x: getattr(gpu, x) for x in ("mate_a", "mate_b", "y_a", "y_b")}
        if gpu.status == "ok":
            break
    final = forced.solve_rounded(kd, 4, n, state=state)
    for x in ("y_a", "y_b"):
        assert np.array_equal(host(getattr(final, x)), orc[x])


def test_explicit_transport_copies_forced_modes(forced):
    """The copies of the transport reduction with the column duals in global
    memory: the plan bit-exact."""
    rng = np.random.default_rng(3)
    C = rng.random((40, 50)).astype(np.float32)
    nu = rng.random(40) + 0.05
    mu = rng.random(50) + 0.05
    nu, mu = nu / nu.sum(), mu / mu.sum()
    orc = oracle.ot_solve(C, nu, mu, 0.1)
    gpu = forced.ot_solve(dev(C), dev(nu), dev(mu), 0.1)
    assert np.array_equal(host(gpu.plan), orc["plan"])
    assert gpu.stats["phases"] == orc["stats"]["phases"]


def test_wide_rows_reject_large_duals(forced):
    """With 18-bit rows the duals travel in 14 bits: an eps whose K + 2 does
    not fit is refused for point sets (K known)."""
    import paper_2203_03732_amd as prot
    X, Y = synth.uniform_points(50, 2, seed=1)
    with pytest.raises(prot.ProtError, match="unsupported"):
        forced.solve_points(dev(X), dev(Y), 1.0 / 20000)


@pytest.mark.parametrize("shift", [0.0, 0.5])
def test_points_150000_d2_full_size(ctx, shift):
    """150,000 points in the unit square (the demand cloud shifted right by
    `shift`), eps = 0.01, costs recomputed in the scan: 300 KB of column
    duals (beyond LDS) and rows beyond 17 bits. Unshifted, nearly every
    nearest neighbour rounds to k = 0 and one phase suffices; shifted, the
    phases compete for the near columns. The certificate: the maximum against
    the pairs of the two convex hulls, every matched pair's rounded cost from
    the oracle (eq. (3) on M), (I1), (I2) on sampled full rows, Sigma k, the
    free rows within the stop threshold, and c(M) <= eps (Sigma y - n) +
    3 eps n."""
    from scipy.spatial import ConvexHull
    n, d, eps = 150000, 2, 0.01
    X, Y = synth.uniform_points(n, d, seed=7)
    Y = np.ascontiguousarray(Y + np.array([shift, 0.0], np.float32))
    Xd, Yd = dev(X), dev(Y)
    print(f"n=150000 d=2 shift={shift} on the fly", flush=True)
    loop = ctx.solve_points(Xd, Yd, eps, complete=False)
    full = ctx.solve_points(Xd, Yd, eps)
    m = np.float32(loop.stats["cost_scale"])
    hx, hy = ConvexHull(X).vertices, ConvexHull(Y).vertices
    bi, ai = np.repeat(hx, len(hy)), np.tile(hy, len(hx))
    d2 = ((X[bi].astype(np.float64) - Y[ai]) ** 2).sum(1)
    hull_max = d2.max()
    assert hull_max * (1 - 2.0 ** -20) <= float(m) <= hull_max * (1 + 2.0 ** -20)
    mate_a, mate_b = host(loop.mate_a), host(loop.mate_b)
    ya, yb = host(loop.y_a).astype(np.int64), host(loop.y_b).astype(np.int64)
    matched = np.nonzero(mate_b >= 0)[0]
    assert np.array_equal(mate_a[mate_b[matched]], matched)
    assert n - len(matched) <= oracle.threshold(eps, n)
    assert (yb >= 0).all() and (ya <= 0).all() and (ya[mate_a < 0] == 0).all()
    kp = oracle.points_pairs_f32(X, Y, eps, m, matched, mate_b[matched]).astype(np.int64)
    assert np.array_equal(ya[mate_b[matched]] + yb[matched], kp)  # eq. (3) on M
    assert loop.stats["sum_k"] == kp.sum()
    rng = np.random.default_rng(2)
    cols = np.arange(n)
    for b in rng.choice(n, 8, replace=False):
        kr = oracle.points_pairs_f32(X, Y, eps, m, np.full(n, b), cols).astype(np.int64)
        assert (ya + yb[b] <= kr + 1).all(), f"(I2) fails on row {b}"  # eq. (2)
    for x in ("y_a", "y_b"):
        assert torch.equal(getattr(loop, x), getattr(full, x))
    assert (host(full.mate_b) >= 0).all()
    lb = eps * (ya.sum() + yb.sum() - n)
    assert full.stats["cost"] <= lb + 3 * eps * n + 1e-9
    print(f"n=150000 shift={shift}: {full.stats['phases']} phases, "
          f"loop {full.stats['ms_loop_kernel']:.1f} ms", flush=True)
