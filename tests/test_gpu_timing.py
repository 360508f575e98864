"""Timing of solves enqueued without statistics: prot_loop_times returns the
device times of the last phase-loop launches (events carried by the
launches), the same values the statistics of a solve report."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_loop_times_of_enqueued_solves():
    import paper_2203_03732_amd as prot
    from paper_2203_03732_amd import synth
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    X, Y = synth.uniform_points(3000, 2, seed=4)
    Xd, Yd = torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda()
    ctx = prot.Context(0)
    try:
        assert len(ctx.loop_times(5)) == 0  # nothing launched yet
        for _ in range(3):
            ctx.solve_points(Xd, Yd, 0.02, stats=False)
        assert ctx.status() == "ok"
        t = ctx.loop_times(5)
        assert len(t) == 3 and (t > 0).all() and (t < 1e3).all()
        r = ctx.solve_points(Xd, Yd, 0.02)
        last = ctx.loop_times(1)
        assert len(last) == 1 and last[0] == pytest.approx(r.stats["ms_loop_kernel"], rel=1e-6)
        assert len(ctx.loop_times(0)) == 0
        # the same deterministic solve: times of one size
        t4 = ctx.loop_times(4)
        assert len(t4) == 4 and t4.max() < 5 * t4.min()
    finally:
        torch.cuda.synchronize()
        ctx.close()
