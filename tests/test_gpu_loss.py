"""GPU parity of the matching-based OT loss and its hand-written backward:
forward and gradients against the oracle's closed form on the oracle's
(identical) matching, the exact-plan gradient and finite differences of the
exact OT cost on tiny generic inputs, and autograd plumbing."""
import itertools
import math

import numpy as np
import pytest

import oracle
from paper_2203_03732_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def prot():
    import paper_2203_03732_amd as p
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return p


def oracle_matching(X, Y, eps):
    k, _ = oracle.round_points_f32(X, Y, eps)
    return oracle.solve_rounded(k, oracle.threshold(eps, X.shape[0]))


def test_loss_and_grad_match_oracle(prot):
    batch, n, d, eps = 6, 300, 8, 0.02
    X, Y = synth.shifted_gaussian_batch(batch, n, d, 0.5, seed=2)
    Xd = torch.from_numpy(X).cuda().requires_grad_(True)
    Yd = torch.from_numpy(Y).cuda().requires_grad_(True)
    loss = prot.ot_match_loss(Xd, Yd, eps)
    g = torch.linspace(0.5, 2.0, batch, device="cuda")
    (loss * g).sum().backward()
    for i in range(batch):
        ref = oracle_matching(X[i], Y[i], eps)
        want = oracle.ot_loss(X[i], Y[i], ref["mate_b"])
        assert math.isclose(float(loss[i]), want, rel_tol=1e-6)
        dX, dY = oracle.ot_loss_grad(X[i], Y[i], ref["mate_b"], float(g[i]))
        np.testing.assert_allclose(Xd.grad[i].cpu().numpy(), dX, rtol=1e-5, atol=1e-6)
        np.testing.assert_allclose(Yd.grad[i].cpu().numpy(), dY, rtol=1e-5, atol=1e-6)


def _exact(X, Y):
    n = X.shape[0]
    best = None
    for perm in itertools.permutations(range(n)):
        v = sum(float(((X[b] - Y[perm[b]]) ** 2).sum()) for b in range(n)) / n
        if best is None or v < best[0]:
            best = (v, np.array(perm))
    return best


@pytest.mark.parametrize("seed", range(3))
def test_gradient_is_exact_plan_gradient_and_finite_differences(prot, seed):
    """Tiny generic inputs with eps small enough that 3 eps n is below the
    optimality gap (normalised): the solver's matching is the exact optimum,
    and the backward equals central differences of the exact OT cost."""
    rng = np.random.default_rng(seed)
    n, d = 6, 2
    X = rng.standard_normal((1, n, d)).astype(np.float32)
    Y = rng.standard_normal((1, n, d)).astype(np.float32)
    X64, Y64 = X[0].astype(np.float64), Y[0].astype(np.float64)
    w, perm = _exact(X64, Y64)
    costs = sorted(sum(float(((X64[b] - Y64[p[b]]) ** 2).sum()) for b in range(n))
                   for p in itertools.permutations(range(n)))
    m = max(float(((X64[b] - Y64[a]) ** 2).sum()) for b in range(n) for a in range(n))
    gap = (costs[1] - costs[0]) / m
    eps = min(0.2, gap / (3 * n + 1))
    Xd = torch.from_numpy(X).cuda().requires_grad_(True)
    Yd = torch.from_numpy(Y).cuda().requires_grad_(True)
    loss = prot.ot_match_loss(Xd, Yd, eps)
    loss.sum().backward()
    assert math.isclose(float(loss[0]), w, rel_tol=1e-5)
    dX, dY = oracle.ot_loss_grad(X64, Y64, perm)
    np.testing.assert_allclose(Xd.grad[0].cpu().numpy(), dX, rtol=1e-4, atol=1e-5)
    np.testing.assert_allclose(Yd.grad[0].cpu().numpy(), dY, rtol=1e-4, atol=1e-5)
    h = 1e-4
    for M, G in ((X64, Xd.grad[0]), (Y64, Yd.grad[0])):
        G = G.cpu().numpy()
        for idx in np.ndindex(M.shape):
            old = M[idx]
            M[idx] = old + h
            wp = _exact(X64, Y64)[0]
            M[idx] = old - h
            wm = _exact(X64, Y64)[0]
            M[idx] = old
            assert abs((wp - wm) / (2 * h) - G[idx]) < 1e-4


def _oracle_runs(X, Y, eps):
    """The oracle on every instance; the C oracle releases the GIL, so the
    instances run on parallel host threads (each one single-threaded)."""
    import os
    from concurrent.futures import ThreadPoolExecutor
    workers = max(1, min(16, os.cpu_count() or 1))
    with ThreadPoolExecutor(workers) as ex:
        return list(ex.map(lambda i: oracle_matching(X[i], Y[i], eps), range(X.shape[0])))


def test_shifted_gaussians_64x2048_d64(prot):
    """64 instances, n = 2048, X ~ N(0, I_64), Y ~ N(0.5, I_64), eps = 0.01:
    forward + backward as the benchmark runs them. Every instance's matching,
    duals and statistics equal the oracle's; every loss, dX and dY equal the
    closed form on the oracle's matching."""
    batch, n, d, eps = 64, 2048, 64, 0.01
    X, Y = synth.shifted_gaussian_batch(batch, n, d, 0.5, seed=0)
    Xd = torch.from_numpy(X).cuda().requires_grad_(True)
    Yd = torch.from_numpy(Y).cuda().requires_grad_(True)
    loss = prot.ot_match_loss(Xd, Yd, eps)
    loss.sum().backward()
    plan = prot.context().cached_batch([n] * batch, d, eps, eps_mode="algorithmic")
    mb = plan.mate_b.cpu().numpy().reshape(batch, n)
    ma = plan.mate_a.cpu().numpy().reshape(batch, n)
    ya = plan.y_a.cpu().numpy().reshape(batch, n)
    yb = plan.y_b.cpu().numpy().reshape(batch, n)
    stats = plan.stats()
    refs = _oracle_runs(X, Y, eps)
    gX, gY = Xd.grad.cpu().numpy(), Yd.grad.cpu().numpy()
    for i, ref in enumerate(refs):
        for name, arr in (("mate_b", mb), ("mate_a", ma), ("y_a", ya), ("y_b", yb)):
            assert np.array_equal(arr[i], ref[name]), f"instance {i}: {name}"
        for s in ("phases", "sum_free", "rounds", "max_rounds", "scanned", "sum_k",
                  "completed_pairs"):
            assert stats[i][s] == ref["stats"][s], f"instance {i}: {s}"
        want = oracle.ot_loss(X[i], Y[i], ref["mate_b"])
        assert math.isclose(float(loss[i]), want, rel_tol=1e-6)
        dX, dY = oracle.ot_loss_grad(X[i], Y[i], ref["mate_b"])
        np.testing.assert_allclose(gX[i], dX, rtol=1e-5, atol=1e-7)
        np.testing.assert_allclose(gY[i], dY, rtol=1e-5, atol=1e-7)


@pytest.mark.parametrize("batch,n,d", [(1, 1, 1), (3, 257, 5), (16, 1000, 64)])
def test_standalone_loss_calls(prot, batch, n, d):
    """prot_ot_loss_fwd/bwd without a batch plan, on the oracle's matchings
    (and on a partial matching with unmatched rows): the loss and both
    gradients against the closed form; the gradients bit-equal to the plan's
    backward on the same matching."""
    eps = 0.05
    X, Y = synth.shifted_gaussian_batch(batch, n, d, 0.5, seed=n + d)
    mates = np.stack([oracle_matching(X[i], Y[i], eps)["mate_b"] for i in range(batch)])
    if n > 1:
        mates[0, ::3] = -1  # a partial matching
    ctx = prot.context()
    Xd, Yd = torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda()
    md = torch.from_numpy(mates).cuda()
    g = torch.linspace(0.5, 2.0, batch, device="cuda")
    loss = ctx.ot_loss(Xd, Yd, md)
    dX, dY = ctx.ot_loss_grad(Xd, Yd, md, g)
    for i in range(batch):
        assert math.isclose(float(loss[i]), oracle.ot_loss(X[i], Y[i], mates[i]), rel_tol=1e-6,
                            abs_tol=1e-30)
        wX, wY = oracle.ot_loss_grad(X[i], Y[i], mates[i], float(g[i]))
        np.testing.assert_allclose(dX[i].cpu().numpy(), wX, rtol=1e-5, atol=1e-7)
        np.testing.assert_allclose(dY[i].cpu().numpy(), wY, rtol=1e-5, atol=1e-7)
    plan = ctx.cached_batch([n] * batch, d, eps)
    inv = np.full_like(mates, -1)
    for i in range(batch):
        rows = np.nonzero(mates[i] >= 0)[0]
        inv[i, mates[i, rows]] = rows
    pX, pY = plan.loss_grad(Xd.view(batch * n, d), Yd.view(batch * n, d), g,
                            torch.from_numpy(inv.reshape(-1)).cuda(), md.view(-1))
    assert torch.equal(pX.view(batch, n, d), dX) and torch.equal(pY.view(batch, n, d), dY)
    assert torch.equal(plan.loss(Xd.view(batch * n, d), Yd.view(batch * n, d), md.view(-1)), loss)
