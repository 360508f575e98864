"""A point-set solve whose loop recomputes its costs hands over to the stored
matrix after a number of rounds (PROT_AUTO_SWITCH_ROUNDS forces the round
here; by default it follows the matrix's size): the loop stops at a phase
start, the matrix is built and the loop resumes from the state reached. The
result — matching, duals, every statistic and the per-phase record — is the
oracle's, as for one run (Section 2.2; the trajectory does not depend on
where the costs come from)."""
import os

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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.cpu().numpy()


def _solve(ctx, X, Y, eps, switch):
    old = os.environ.get("PROT_AUTO_SWITCH_ROUNDS")
    os.environ["PROT_AUTO_SWITCH_ROUNDS"] = str(switch)
    try:
        launches = len(ctx.loop_times(1024))
        r = ctx.solve_points(dev(X), dev(Y), eps, storage="on_the_fly")
        parts = len(ctx.loop_times(1024)) - launches
    finally:
        if old is None:
            del os.environ["PROT_AUTO_SWITCH_ROUNDS"]
        else:
            os.environ["PROT_AUTO_SWITCH_ROUNDS"] = old
    return r, parts


def _same(gpu, orc, what, ctx):
    for x in ("mate_a", "mate_b", "y_a", "y_b"):
        g = host(getattr(gpu, x))
        assert np.array_equal(g, orc[x]), f"{what}: {x} differs at {np.nonzero(g != orc[x])[0][:10]}"
    for s in STAT_KEYS:
        assert gpu.stats[s] == orc["stats"][s], f"{what}: stat {s} {gpu.stats[s]} != {orc['stats'][s]}"
    assert np.array_equal(ctx.trace(), orc["trace"]), f"{what}: per-phase record differs"


@pytest.mark.parametrize("switch", [1, 4, 9, 30])
def test_handover_square(ctx, switch):
    X, Y = synth.uniform_points(2000, 2, seed=5)
    Y = np.ascontiguousarray(Y + np.array([0.3, 0.0], np.float32))
    print(f"hand-over n=2000 after round {switch}", flush=True)
    orc = oracle.solve_points(X, Y, 0.01, trace=True)
    gpu, parts = _solve(ctx, X, Y, 0.01, switch)
    assert gpu.status == "ok"
    _same(gpu, orc, f"switch {switch}", ctx)
    # the loop ran in two launches unless it ended before the round
    assert parts == (2 if orc["stats"]["rounds"] > switch + 2 else parts)
    assert parts in (1, 2)


def test_handover_rect_d3(ctx):
    X, Y = synth.uniform_points(700, 3, seed=6, n_a=1500)
    X = np.ascontiguousarray(X * np.float32(0.5))  # rows crowd one corner
    print("hand-over 700 x 1500, d = 3", flush=True)
    orc = oracle.solve_points(X, Y, 0.02, trace=True)
    assert orc["stats"]["phases"] > 2
    gpu, parts = _solve(ctx, X, Y, 0.02, 1)
    assert gpu.status == "ok" and parts == 2
    _same(gpu, orc, "rect d=3", ctx)


def test_handover_n10000(ctx):
    """The 10,000-point plane instance handing over after phase 0."""
    X, Y = synth.uniform_points(10000, 2, seed=0)
    print("hand-over n=10000", flush=True)
    orc = oracle.solve_points(X, Y, 0.01, trace=True)
    gpu, parts = _solve(ctx, X, Y, 0.01, 15)
    assert gpu.status == "ok" and parts == 2
    _same(gpu, orc, "n=10000", ctx)


def test_handover_without_room_for_the_matrix(ctx):
    """When the matrix cannot be allocated the loop resumes recomputing its
    costs (PROT_HANDOVER_NO_MATRIX takes that path on purpose): the same
    result in two launches."""
    X, Y = synth.uniform_points(1500, 2, seed=8)
    Y = np.ascontiguousarray(Y + np.array([0.0, 0.4], np.float32))
    orc = oracle.solve_points(X, Y, 0.01, trace=True)
    os.environ["PROT_HANDOVER_NO_MATRIX"] = "1"
    try:
        gpu, parts = _solve(ctx, X, Y, 0.01, 2)
    finally:
        del os.environ["PROT_HANDOVER_NO_MATRIX"]
    assert gpu.status == "ok" and parts == 2
    _same(gpu, orc, "no matrix", ctx)
