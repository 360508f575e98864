"""GPU parity for the cost variants of Section 5 (plain Euclidean; half the L1
distance of vectors normalised to sum 1): rounded costs bit-exact with the
oracle's definitions, and whole solves bit-exact with the oracle's loop on
those costs."""
import math

import numpy as np
import pytest

import oracle
from paper_2203_03732_amd import synth
from invariants import check_I1

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

STAT_KEYS = ("phases", "sum_free", "rounds", "max_rounds", "scanned", "sum_k")


@pytest.fixture(scope="module")
def ctx():
    import paper_2203_03732_amd as prot
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = prot.Context(0)
    yield c
    torch.cuda.synchronize()
    c.set_cost_metric("sqeuclidean")
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.cpu().numpy()


def _images(n, seed, d=784):
    if d == 784:
        return synth.digit_images(n, seed=seed)
    rng = np.random.default_rng(seed)
    X = rng.random((n, d)).astype(np.float32)
    X[X < 0.5] = 0.0
    X[:, 0] += 0.25  # every vector has a positive sum
    return X


@pytest.mark.parametrize("n_b,n_a,d,eps", [(1, 9, 2, 0.1), (300, 301, 2, 0.01),
                                           (1000, 1000, 3, 0.005), (333, 500, 16, 0.02),
                                           (97, 130, 784, 0.05)])
def test_build_euclidean_bit_exact(ctx, n_b, n_a, d, eps):
    X, Y = synth.uniform_points(n_b, d, seed=n_b + d, n_a=n_a)
    ctx.set_cost_metric("euclidean")
    try:
        k, m = ctx.build_costs(dev(X), dev(Y), eps)
        torch.cuda.synchronize()
    finally:
        ctx.set_cost_metric("sqeuclidean")
    ko, mo = oracle.round_points_euclid_f32(X, Y, eps)
    assert float(host(m)[0]) == mo
    assert np.array_equal(host(k)[:, :n_a], ko)


@pytest.mark.parametrize("n_b,n_a,d,eps", [(1, 5, 4, 0.25), (200, 250, 784, 0.1),
                                           (130, 70, 784, 0.01), (301, 299, 16, 0.05),
                                           (64, 64, 2, 0.1)])
def test_build_l1_bit_exact(ctx, n_b, n_a, d, eps):
    X, Y = _images(n_b, 1, d), _images(n_a, 2, d)
    ctx.set_cost_metric("l1_normalized")
    try:
        k, m = ctx.build_costs(dev(X), dev(Y), eps)
        torch.cuda.synchronize()
    finally:
        ctx.set_cost_metric("sqeuclidean")
    assert float(host(m)[0]) == 2.0
    assert np.array_equal(host(k)[:, :n_a], oracle.round_l1_normalized_f32(X, Y, eps))


def _solve_case(ctx, metric, X, Y, eps, origin="diag"):
    ctx.set_cost_metric(metric)
    try:
        gpu = ctx.solve_points(dev(X), dev(Y), eps, origin=origin)
    finally:
        ctx.set_cost_metric("sqeuclidean")
    if metric == "euclidean":
        k, m = oracle.round_points_euclid_f32(X, Y, eps)
    else:
        k = oracle.round_l1_normalized_f32(X, Y, eps)
    orc = oracle.solve_rounded(k, oracle.threshold(eps, X.shape[0]), origin=origin)
    for x in ("mate_a", "mate_b", "y_a", "y_b"):
        assert np.array_equal(host(getattr(gpu, x)), orc[x]), f"{metric}: {x}"
    for s in STAT_KEYS:
        assert gpu.stats[s] == orc["stats"][s], f"{metric}: {s}"
    mb = orc["mate_b"]
    X64, Y64 = X.astype(np.float64), Y.astype(np.float64)
    if metric == "euclidean":
        d2 = ((X64 - Y64[mb]) ** 2).sum(1)
        want = float(np.sqrt(d2).sum()) / math.sqrt(m)
        assert gpu.stats["cost_scale"] == m
    else:
        Xh = X64 / X64.sum(1, keepdims=True)
        Yh = Y64 / Y64.sum(1, keepdims=True)
        want = float(0.5 * np.abs(Xh - Yh[mb]).sum())
        assert gpu.stats["cost_scale"] == 2.0
    assert math.isclose(gpu.stats["cost"], want, rel_tol=1e-12)
    return gpu, orc


@pytest.mark.parametrize("origin", ["diag", "zero"])
def test_solve_euclidean(ctx, origin):
    X, Y = synth.uniform_points(2000, 2, seed=12)
    _solve_case(ctx, "euclidean", X, Y, 0.01, origin)


@pytest.mark.parametrize("origin", ["diag", "zero"])
@pytest.mark.parametrize("eps", [0.5, 0.1])
def test_solve_l1_images(ctx, eps, origin):
    X, Y = synth.digit_images(1000, seed=21), synth.digit_images(1000, seed=22)
    _solve_case(ctx, "l1_normalized", X, Y, eps, origin)


def test_solve_metrics_rectangular(ctx):
    X, Y = synth.uniform_points(700, 3, seed=5, n_a=900)
    _solve_case(ctx, "euclidean", X, Y, 0.02)
    X, Y = synth.digit_images(300, seed=6), synth.digit_images(450, seed=7)
    _solve_case(ctx, "l1_normalized", X, Y, 0.1)


def test_euclidean_full_size_n10000(ctx):
    """Section 5's synthetic experiment at n = 10,000, eps = 0.01, with the
    plain Euclidean cost: whole solve against the oracle."""
    X, Y = synth.uniform_points(10000, 2, seed=0)
    gpu, orc = _solve_case(ctx, "euclidean", X, Y, 0.01)
    assert gpu.stats["phases"] == orc["stats"]["phases"]


def test_l1_images_full_size_sampled(ctx):
    """Section 5's image experiment at n = 10,000 (784-pixel stand-ins),
    eps = 0.1: the GPU's rounded costs on 300 sampled rows x 300 sampled
    columns equal the oracle's (each entry depends on its two images only);
    the solve's duals satisfy (I1) and (I2) on the sampled rows."""
    n, eps = 10000, 0.1
    X, Y = synth.digit_images(n, seed=31), synth.digit_images(n, seed=32)
    Xd, Yd = dev(X), dev(Y)
    ctx.set_cost_metric("l1_normalized")
    try:
        k, _ = ctx.build_costs(Xd, Yd, eps)
        gpu = ctx.solve_points(Xd, Yd, eps)
        torch.cuda.synchronize()
    finally:
        ctx.set_cost_metric("sqeuclidean")
    rng = np.random.default_rng(0)
    rows = np.sort(rng.choice(n, 300, replace=False))
    cols = np.sort(rng.choice(n, 300, replace=False))
    ks = host(k[torch.from_numpy(rows).cuda()][:, torch.from_numpy(cols).cuda()])
    assert np.array_equal(ks, oracle.round_l1_normalized_f32(X[rows], Y[cols], eps))
    kr = host(k[torch.from_numpy(rows).cuda()])[:, :n]
    ya, yb = host(gpu.y_a), host(gpu.y_b)
    check_I1(host(gpu.mate_a), ya, yb)
    S = yb[rows][:, None].astype(np.int64) + ya[None, :]
    assert (S <= kr + 1).all(), "eq. (2) on sampled rows"
    assert gpu.stats["completed_pairs"] <= oracle.threshold(eps, n)


def test_metric_rejections(ctx):
    import paper_2203_03732_amd as prot
    X, Y = synth.uniform_points(50, 2, seed=1)
    ctx.set_cost_metric("euclidean")
    try:
        with pytest.raises(prot.ProtError) as e:
            ctx.solve_points(dev(X), dev(Y), 0.1, storage="on_the_fly")
        assert e.value.name == "unsupported"
        ctx.set_cost_metric("l1_normalized")
        bad = X.copy()
        bad[3, 1] = -0.5
        with pytest.raises(prot.ProtError) as e:
            ctx.solve_points(dev(bad), dev(Y), 0.1)
        assert e.value.name == "range"
        bad = X.copy()
        bad[7] = 0.0
        with pytest.raises(prot.ProtError) as e:
            ctx.build_costs(dev(X), dev(bad), 0.1)
        assert e.value.name == "range"
    finally:
        ctx.set_cost_metric("sqeuclidean")
    with pytest.raises(KeyError):
        ctx.set_cost_metric("cosine")
    assert ctx._lib.prot_set_cost_metric(ctx._h, 7) == -1  # PROT_E_ARG
