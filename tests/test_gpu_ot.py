"""GPU parity for optimal transport through copies (Section 4): the HIP
path, through the C ABI, against the CPU oracle on the same inputs. The plan
and the repaired mass must be bit-exact, the duals (in the two-cluster form
of Lemma 4.1) and the phase-loop statistics equal; the plan's cost agrees to
rounding order."""
import math

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


def _clusters(y, owners_counts):
    """Per point: the smaller dual of its copies and how many hold it."""
    lo, nlo, i = [], [], 0
    for c in owners_counts:
        v = y[i:i + c]
        i += c
        if c == 0:
            lo.append(0)
            nlo.append(0)
        else:
            lo.append(int(v.min()))
            nlo.append(int((v == v.min()).sum()))
    return np.array(lo, np.int32), np.array(nlo, np.int32)


def _compare(gpu, orc, what, plan=True):
    st = gpu.stats
    assert st["theta"] == orc["theta"], what
    assert st["copies_b"] == len(orc["mate_b"]) and st["copies_a"] == len(orc["mate_a"]), what
    for k in STAT_KEYS:
        want = orc["T"] if k == "threshold" else orc["stats"][k]
        assert st[k] == want, f"{what}: stat {k} {st[k]} != {want}"
    lo, nlo = _clusters(orc["y_b"], orc["s"])
    assert np.array_equal(host(gpu.y_b_lo), lo) and np.array_equal(host(gpu.y_b_nlo), nlo), what
    lo, nlo = _clusters(orc["y_a"], orc["d"])
    assert np.array_equal(host(gpu.y_a_lo), lo) and np.array_equal(host(gpu.y_a_nlo), nlo), what
    if plan:
        P = host(gpu.plan)
        assert np.array_equal(P, orc["plan"]), \
            f"{what}: plan differs at {np.argwhere(P != orc['plan'])[:5].tolist()}"
        assert st["repaired_mass"] == orc["repaired"], what
        assert math.isclose(st["cost"], orc["cost"], rel_tol=1e-12, abs_tol=1e-15), what


def _instance(n_b, n_a, seed, zeros=0, points=False, shift=0.0):
    if points:
        from paper_2203_03732_amd import synth
        return synth.transport_clouds(n_b, n_a, seed=seed, shift=shift)
    rng = np.random.default_rng(seed)
    C = rng.random((n_b, n_a)).astype(np.float32)
    return C, _masses(rng, n_b, zeros), _masses(rng, n_a)


@pytest.mark.parametrize("origin", ["diag", "zero"])
@pytest.mark.parametrize("n_b,n_a,eps,seed,zeros", [
    (1, 1, 0.1, 0, 0), (5, 7, 0.1, 1, 0), (9, 4, 0.2, 2, 1), (40, 40, 0.05, 3, 3),
    (100, 150, 0.05, 4, 0), (257, 130, 0.1, 5, 7), (300, 300, 0.02, 6, 0)])
def test_ot_bit_exact(ctx, n_b, n_a, eps, seed, zeros, origin):
    C, nu, mu = _instance(n_b, n_a, seed, zeros)
    orc = oracle.ot_solve(C, nu, mu, eps, origin=origin)
    gpu = ctx.ot_solve(dev(C), dev(nu), dev(mu), eps, origin=origin)
    assert gpu.status == "ok" and orc["status"] == "ok"
    _compare(gpu, orc, f"{n_b}x{n_a} eps={eps} seed={seed} {origin}")


def test_ot_points_shifted_clouds(ctx):
    """Two 1,000-point clouds in the plane, the demand one shifted by 1,
    random masses, eps = 0.1 (the transport workload of the benchmark)."""
    C, nu, mu = _instance(1000, 1000, 11, points=True, shift=1.0)
    orc = oracle.ot_solve(C, nu, mu, 0.1)
    gpu = ctx.ot_solve(dev(C), dev(nu), dev(mu), 0.1)
    _compare(gpu, orc, "clouds")
    assert orc["stats"]["phases"] > 5


@pytest.mark.parametrize("eps_mode", ["algorithmic", "strict"])
def test_ot_eps_modes(ctx, eps_mode):
    C, nu, mu = _instance(60, 50, 21, points=True, shift=0.5)
    gpu = ctx.ot_solve(dev(C), dev(nu), dev(mu), 0.3, eps_mode=eps_mode)
    ei = 0.3 / 3 if eps_mode == "strict" else 0.3  # the library divides the same way
    orc = oracle.ot_solve(C, nu, mu, ei)
    assert gpu.stats["eps_internal"] == pytest.approx(ei, rel=1e-15)
    _compare(gpu, orc, eps_mode)


def test_ot_forced_plans(ctx):
    rng = np.random.default_rng(3)
    C = rng.random((1, 9)).astype(np.float32)
    mu = _masses(rng, 9, zeros=2)
    gpu = ctx.ot_solve(dev(C), dev(np.array([1.0])), dev(mu), 0.1)
    assert np.allclose(host(gpu.plan)[0], mu, rtol=0, atol=1e-12)
    C = rng.random((7, 1)).astype(np.float32)
    nu = _masses(rng, 7)
    gpu = ctx.ot_solve(dev(C), dev(nu), dev(np.array([1.0])), 0.2)
    assert np.allclose(host(gpu.plan)[:, 0], nu, rtol=0, atol=1e-12)


def test_ot_partial(ctx):
    """Stopped after two phases: duals and statistics as the oracle's state
    after two phases (no completion)."""
    C, nu, mu = _instance(50, 60, 8, points=True, shift=1.0)
    orc = oracle.ot_solve(C, nu, mu, 0.1, max_phases=2)
    assert orc["status"] == "partial"
    gpu = ctx.ot_solve(dev(C), dev(nu), dev(mu), 0.1, max_phases=2)
    assert gpu.status == "partial"
    _compare(gpu, orc, "partial", plan=False)


def test_ot_rejects(ctx):
    import paper_2203_03732_amd as prot
    C = np.full((3, 2), 0.5, np.float32)
    with pytest.raises(prot.ProtError) as e:
        ctx.ot_solve(dev(C), dev(np.array([0.5, 0.3, 0.1])), dev(np.array([0.5, 0.5])), 0.1)
    assert e.value.name == "range"
    with pytest.raises(prot.ProtError) as e:
        ctx.ot_solve(dev(C), dev(np.array([0.5, 0.7, -0.2])), dev(np.array([0.5, 0.5])), 0.1)
    assert e.value.name == "range"
    C[1, 1] = 1.5
    with pytest.raises(prot.ProtError) as e:
        ctx.ot_solve(dev(C), dev(np.array([0.5, 0.3, 0.2])), dev(np.array([0.5, 0.5])), 0.1)
    assert e.value.name == "range"
    # theta = 4 * 1000 / 0.01 = 400,000 demand copies: beyond the LDS dual array
    C = np.full((1000, 10), 0.5, np.float32)
    with pytest.raises(prot.ProtError) as e:
        ctx.ot_solve(dev(C), dev(np.full(1000, 1e-3)), dev(np.full(10, 0.1)), 0.01)
    assert e.value.name == "unsupported"


def test_ot_repeat_and_then_assignment(ctx):
    """Two transport solves of different shapes in a row, then a plain
    assignment solve on the same context: workspaces are resized and every
    result still equals the oracle's."""
    from paper_2203_03732_amd import synth
    for n_b, n_a, seed in [(120, 80, 31), (30, 200, 32)]:
        C, nu, mu = _instance(n_b, n_a, seed)
        orc = oracle.ot_solve(C, nu, mu, 0.1)
        _compare(ctx.ot_solve(dev(C), dev(nu), dev(mu), 0.1), orc, f"repeat {n_b}x{n_a}")
    X, Y = synth.uniform_points(700, 2, seed=5)
    gpu = ctx.solve_points(dev(X), dev(Y), 0.02)
    k, _ = oracle.round_points_f32(X, Y, 0.02)
    ref = oracle.solve_rounded(k, oracle.threshold(0.02, 700))
    assert np.array_equal(host(gpu.mate_b), ref["mate_b"])
    assert np.array_equal(host(gpu.y_b), ref["y_b"])
