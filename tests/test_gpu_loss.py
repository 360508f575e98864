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


def test_shifted_gaussians_64x2048_d64(prot):
    """64 instances, n = 2048, X ~ N(0, I_64), Y ~ N(0.5, I_64), eps = 0.01:
    forward + backward. Two instances are checked bit for bit against the
    oracle's matching; every instance's loss and gradient against the closed
    form on the GPU's matching, which must be a permutation."""
    batch, n, d, eps = 64, 2048, 64, 0.01
    X, Y = synth.shifted_gaussian_batch(batch, n, d, 0.5, seed=0)
    Xd = torch.from_numpy(X).cuda().requires_grad_(True)
    Yd = torch.from_numpy(Y).cuda().requires_grad_(True)
    loss = prot.ot_match_loss(Xd, Yd, eps)
    loss.sum().backward()
    plan = prot.context().cached_batch([n] * batch, d, eps, eps_mode="algorithmic")
    mb = plan.mate_b.cpu().numpy().reshape(batch, n)
    for i in (0, 37):
        ref = oracle_matching(X[i], Y[i], eps)
        assert np.array_equal(mb[i], ref["mate_b"]), f"instance {i}"
    gX, gY = Xd.grad.cpu().numpy(), Yd.grad.cpu().numpy()
    for i in range(batch):
        assert np.array_equal(np.sort(mb[i]), np.arange(n))
        want = oracle.ot_loss(X[i], Y[i], mb[i])
        assert math.isclose(float(loss[i]), want, rel_tol=1e-6)
        Ym = Y[i].astype(np.float64)[mb[i]]
        np.testing.assert_allclose(gX[i], 2.0 * (X[i] - Ym) / n, rtol=1e-5, atol=1e-7)
