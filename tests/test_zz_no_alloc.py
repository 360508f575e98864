"""The context-free loss forward that allocates nothing
(prot_ot_loss_fwd_static, partial sums in the library's fixed device array)
against the context entry point prot_ot_loss_fwd: bit-identical losses on two
calls in a row, the second with a smaller input, and a clear error beyond the
array's size."""
import ctypes

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def inputs(batch, n, d, seed):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((batch, n, d), dtype=np.float32)
    Y = (rng.standard_normal((batch, n, d), dtype=np.float32) + 0.5).astype(np.float32)
    mate = np.stack([rng.permutation(n) for _ in range(batch)]).astype(np.int32)
    mate[:, ::7] = -1  # unmatched rows add nothing
    return (torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda(),
            torch.from_numpy(mate).cuda())


def reference_f64(X, Y, mate):
    X, Y, mate = X.cpu().numpy(), Y.cpu().numpy(), mate.cpu().numpy()
    out = []
    for i in range(X.shape[0]):
        m = mate[i]
        rows = np.nonzero(m >= 0)[0]
        diff = X[i, rows].astype(np.float64) - Y[i, m[rows]].astype(np.float64)
        out.append((diff * diff).sum() / X.shape[1])
    return np.array(out)


def test_static_loss_matches_the_context_call_twice():
    import paper_2203_03732_amd as prot
    ctx = prot.Context(0)
    try:
        for batch, n, d, seed in ((16, 2048, 64, 1), (3, 300, 5, 2)):
            X, Y, mate = inputs(batch, n, d, seed)
            print(f"static loss: batch={batch} n={n} d={d} seed={seed}", flush=True)
            want = ctx.ot_loss(X, Y, mate)
            got = prot._lib.ot_loss_static(X, Y, mate)
            torch.cuda.synchronize()
            assert torch.equal(got, want), (got, want)
            ref = reference_f64(X, Y, mate)
            np.testing.assert_allclose(got.cpu().numpy(), ref, rtol=1e-6)
    finally:
        torch.cuda.synchronize()
        ctx.close()


def test_static_loss_rejects_sizes_beyond_its_array():
    import paper_2203_03732_amd as prot
    lib = prot.load()
    dummy = torch.zeros(8, dtype=torch.float32, device="cuda")
    p = ctypes.c_void_p(dummy.data_ptr())
    # 1,100 instances of 10,000 x 64 coordinates: 64 partial sums each
    rc = lib.prot_ot_loss_fwd_static(1100, 10000, 64, p, p, p, p, None)
    assert rc == -8  # PROT_E_UNSUPPORTED, nothing enqueued
    assert b"fixed array holds 65536" in lib.prot_last_error(None)
    assert lib.prot_ot_loss_fwd_static(-1, 10, 2, p, p, p, p, None) == -1
    # the entry point still works afterwards
    X, Y, mate = inputs(2, 100, 3, 5)
    got = prot._lib.ot_loss_static(X, Y, mate)
    torch.cuda.synchronize()
    np.testing.assert_allclose(got.cpu().numpy(), reference_f64(X, Y, mate), rtol=1e-6)
