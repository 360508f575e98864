"""Pins for the CPU oracle against what the paper and the mathematics fix.

None of these compares the oracle with itself: each checks a closed form, an
invariant or bound proved in arXiv:2203.03732, an exact optimum from brute
force or scipy's assignment solver, or exact rational arithmetic.
"""
from fractions import Fraction
import math

import numpy as np
import pytest
from scipy.optimize import linear_sum_assignment

import oracle
from oracle import tiny
from paper_2203_03732_amd import synth
from invariants import (brute_force_opt, check_I1, check_I2, check_matching,
                        check_phase, matching_cost, potential, safe_phase_bounds)


# ---------------------------------------------------------------- eq. (1)

def _exact_floor(c: float, eps_text: str) -> int:
    return math.floor(Fraction(c) / Fraction(eps_text))


@pytest.mark.parametrize("eps_text", ["0.1", "0.01", "0.005", "0.05", "0.3"])
def test_round_cost_matches_exact_rational(eps_text):
    """eq. (1): k = floor(c / eps). Against exact rationals (c is the exact
    float32 value, eps the decimal the caller means), binary64 division may
    differ only where c/eps lies within a few ulps of an integer."""
    eps = float(eps_text)
    C = synth.uniform_costs(300, seed=3)
    C[0, :6] = [0.0, 1.0, 0.5, 0.3, 0.7, np.float32(0.1)]
    k = oracle.round_cost(C, eps)
    flips = 0
    for c, kk in zip(C.ravel().tolist(), k.ravel().tolist()):
        ex = _exact_floor(c, eps_text)
        if kk != ex:
            flips += 1
            q = Fraction(c) / Fraction(eps_text)
            assert abs(kk - ex) == 1
            assert abs(q - round(q)) < Fraction(1, 1 << 40)
    assert flips <= 3
    assert k[0, 0] == 0 and k[0, 1] == math.floor(1 / eps)
    assert k.max() <= math.floor(1 / eps) and k.min() >= 0


def test_round_cost_known_values():
    C = np.array([[0.0, 0.25, 0.5, 1.0]], np.float32)
    assert oracle.round_cost(C, 0.1).tolist() == [[0, 2, 5, 10]]
    assert oracle.round_cost(C, 0.25).tolist() == [[0, 1, 2, 4]]
    assert oracle.round_cost(C, 0.3).tolist() == [[0, 0, 1, 3]]


@pytest.mark.parametrize("bad", [np.nan, -0.001, 1.001, np.inf])
def test_round_cost_rejects_out_of_range(bad):
    C = np.zeros((4, 4), np.float32)
    C[2, 3] = bad
    with pytest.raises(oracle.OracleError, match="range"):
        oracle.round_cost(C, 0.1)


@pytest.mark.parametrize("eps", [0.0, 1.0, -0.1, 1e-6])
def test_round_cost_rejects_bad_eps(eps):
    with pytest.raises(oracle.OracleError, match="eps"):
        oracle.round_cost(np.zeros((2, 2), np.float32), eps)


# ------------------------------------------------- squared Euclidean costs

def test_points_f32_integer_grid_is_exact():
    """On small integer coordinates every binary32 step is exact, so k must
    equal floor((d2/m)/eps) in exact rationals (up to ulp-level flips of the
    binary64 divisions). Rows are X, columns are Y (n_b != n_a pins it)."""
    rng = np.random.default_rng(5)
    X = rng.integers(0, 9, (7, 3)).astype(np.float32)
    Y = rng.integers(0, 9, (5, 3)).astype(np.float32)
    for eps_text in ["0.1", "0.05", "0.01"]:
        k, m = oracle.round_points_f32(X, Y, float(eps_text))
        assert k.shape == (7, 5)
        d2 = [[int(((X[b] - Y[a]) ** 2).sum()) for a in range(5)] for b in range(7)]
        mx = max(max(r) for r in d2)
        assert m == mx
        for b in range(7):
            for a in range(5):
                q = Fraction(d2[b][a], mx) / Fraction(eps_text)
                ex = math.floor(q)
                if k[b, a] != ex:
                    assert abs(q - round(q)) < Fraction(1, 1 << 40)


@pytest.mark.parametrize("d", [2, 3, 16])
def test_points_f32_within_tolerance_of_f64(d):
    """Every rounded-cost difference between the binary32 definition and the
    binary64 reference is one step, at a rounding boundary."""
    X, Y = synth.uniform_points(200, d, seed=d)
    eps = 0.01
    k32, m32 = oracle.round_points_f32(X, Y, eps)
    c64, k64, m64 = oracle.points_cost_f64(X, Y, eps)
    assert abs(m32 - m64) <= 1e-6 * m64
    # reconstruct the binary32 normalised cost from its definition
    diff = X[:, None, :] - Y[None, :, :]
    assert np.abs(k32.astype(int) - k64.astype(int)).max() <= 1
    flip = k32 != k64
    q = c64[flip] / eps
    assert np.all(np.abs(q - np.round(q)) < 1e-4)
    # brute-force binary64 check of c64 itself
    d2 = (diff.astype(np.float64) ** 2).sum(-1)
    np.testing.assert_allclose(c64, d2 / d2.max(), rtol=0, atol=1e-15)


def test_points_zero_max_gives_zero_costs():
    X = np.ones((3, 2), np.float32)
    k, m = oracle.round_points_f32(X, X.copy(), 0.1)
    assert m == 0.0 and (k == 0).all()


# ------------------------------------------------------ the phase loop

def _run_phase_by_phase(k, T, origin):
    """Drive the oracle one phase at a time and check every phase."""
    n = k.shape[0]
    K = int(k.max()) if k.size else 0
    state = dict(mate_a=np.full(n, -1, np.int32), mate_b=np.full(n, -1, np.int32),
                 y_a=np.zeros(n, np.int32), y_b=np.ones(n, np.int32))
    phases = 0
    sum_free = 0
    while True:
        r = oracle.solve_rounded(k, T, origin=origin, max_phases=1, state=state,
                                 complete=False)
        if r["stats"]["phases"] == 0:
            break
        after = {x: r[x] for x in ("mate_a", "mate_b", "y_a", "y_b")}
        check_matching(after["mate_a"], after["mate_b"])
        check_I1(after["mate_a"], after["y_a"], after["y_b"])
        check_I2(k, after["mate_b"], after["y_a"], after["y_b"])
        sum_free += check_phase(k, state, after)
        # Lemma 3.2 in units: |y| <= K + 2
        assert np.abs(after["y_a"]).max() <= K + 2
        assert np.abs(after["y_b"]).max() <= K + 2
        state = after
        phases += 1
        assert phases <= 10 * n * (K + 3) + 10
    free = int((state["mate_b"] < 0).sum())
    assert free <= T
    return state, phases, sum_free


@pytest.mark.parametrize("origin", ["diag", "zero"])
@pytest.mark.parametrize("seed", range(6))
def test_every_phase_keeps_invariants(origin, seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(2, 40))
    K = int(rng.integers(1, 12))
    k = synth.random_k(n, K, seed=seed)
    T = int(rng.integers(0, max(1, n // 4)))
    state, phases, sum_free = _run_phase_by_phase(k, T, origin)
    full = oracle.solve_rounded(k, T, origin=origin, complete=False)
    # Resuming one phase at a time is the same as one uninterrupted run.
    for x in ("mate_a", "mate_b", "y_a", "y_b"):
        assert np.array_equal(full[x], state[x])
    st = full["stats"]
    assert st["phases"] == phases and st["sum_free"] == sum_free
    # Lemma 3.3 summed: sum n_i = Phi_final - Phi_initial (Phi_initial = n).
    assert sum_free == potential(state["y_a"], state["y_b"]) - n
    bound_free, bound_phases = safe_phase_bounds(n, int(k.max()), T)
    assert sum_free <= bound_free and phases <= bound_phases


def test_c1_shaped_instance_invariants():
    C = synth.uniform_costs(150, seed=11)
    eps = 0.05
    k = oracle.round_cost(C, eps)
    _run_phase_by_phase(k, oracle.threshold(eps, 150), "diag")


def _check_bounds(C, eps, origin="diag"):
    n = C.shape[0]
    k = oracle.round_cost(C, eps)
    T = oracle.threshold(eps, n)
    r = oracle.solve_rounded(k, T, origin=origin)
    check_matching(r["mate_a"], r["mate_b"], perfect=True)
    return k, r


@pytest.mark.parametrize("seed", range(25))
def test_additive_error_against_brute_force(seed):
    """Section 3.1: cost <= OPT + 3 eps n (and + eps n when run with eps/3),
    and Lemma 3.1 on the rounded costs: k(M) <= OPT_k + n before completion."""
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 8))
    C = synth.uniform_costs(n, seed=seed)
    opt = brute_force_opt(C)
    for eps in (0.5, 0.3, 0.2, 0.1, 0.05):
        k, r = _check_bounds(C, eps)
        assert matching_cost(C, r["mate_b"]) <= opt + 3 * eps * n + 1e-9
        k3, r3 = _check_bounds(C, eps / 3)
        assert matching_cost(C, r3["mate_b"]) <= opt + eps * n + 1e-9
        pre = oracle.solve_rounded(k, oracle.threshold(eps, n), complete=False)
        mb = pre["mate_b"]
        ks = sum(int(k[b, mb[b]]) for b in range(n) if mb[b] >= 0)
        opt_k = brute_force_opt(k)
        assert ks <= opt_k + n


@pytest.mark.parametrize("n,eps", [(60, 0.1), (200, 0.05), (300, 0.01)])
def test_additive_error_against_scipy(n, eps):
    C = synth.uniform_costs(n, seed=n)
    rows, cols = linear_sum_assignment(C.astype(np.float64))
    opt = float(C.astype(np.float64)[rows, cols].sum())
    for origin in ("diag", "zero"):
        _, r = _check_bounds(C, eps, origin)
        cost = matching_cost(C, r["mate_b"])
        assert opt - 1e-9 <= cost <= opt + 3 * eps * n


def test_exact_when_eps_below_the_gap():
    """If 3 eps n is below the gap between the best and second-best perfect
    matching, the returned matching must be the unique optimum."""
    rng = np.random.default_rng(7)
    n = 30
    perm = rng.permutation(n)
    C = np.ones((n, n), np.float32)
    C[np.arange(n), perm] = 0.0
    eps = 1.0 / (3 * n + 1)
    _, r = _check_bounds(C, eps)
    assert np.array_equal(r["mate_b"], perm)


# ------------------------------------------------------- closed forms

@pytest.mark.parametrize("origin", ["diag", "zero"])
def test_closed_form_identity_costs(origin):
    """k = 0 on the diagonal, K elsewhere: one phase, one round, the identity,
    y(a) = -1, y(b) = 1."""
    n, K = 17, 9
    k = np.full((n, n), K, np.int16)
    np.fill_diagonal(k, 0)
    r = oracle.solve_rounded(k, 0, origin=origin)
    st = r["stats"]
    assert st["phases"] == 1 and st["rounds"] == 1
    assert np.array_equal(r["mate_b"], np.arange(n))
    assert (r["y_a"] == -1).all() and (r["y_b"] == 1).all()
    assert st["sum_k"] == 0 and st["completed_pairs"] == 0


def test_closed_form_all_zero_costs():
    """All-zero k: the diagonal scan order finishes in one round with the
    identity; scanning every row from column 0 needs one round per column,
    each won by the lowest free row, so b gets column b as well."""
    n = 23
    k = np.zeros((n, n), np.int16)
    rd = oracle.solve_rounded(k, 0, origin="diag")
    rz = oracle.solve_rounded(k, 0, origin="zero")
    assert rd["stats"]["rounds"] == 1 and rd["stats"]["phases"] == 1
    assert rz["stats"]["rounds"] == n and rz["stats"]["phases"] == 1
    assert np.array_equal(rd["mate_b"], np.arange(n))
    assert np.array_equal(rz["mate_b"], np.arange(n))


@pytest.mark.parametrize("k0", [0, 1, 5, 40])
def test_closed_form_single_vertex(k0):
    """n = 1: y(b) climbs one step per phase until y(b) = k + 1."""
    k = np.array([[k0]], np.int16)
    r = oracle.solve_rounded(k, 0)
    assert r["stats"]["phases"] == k0 + 1
    assert r["y_b"][0] == k0 + 1 and r["y_a"][0] == -1 and r["mate_b"][0] == 0


def test_closed_form_threshold_at_least_n():
    k = synth.random_k(9, 5, seed=1)
    r = oracle.solve_rounded(k, 9)
    assert r["stats"]["phases"] == 0 and r["stats"]["completed_pairs"] == 9
    assert np.array_equal(r["mate_b"], np.arange(9))


def test_empty_instance():
    r = oracle.solve_rounded(np.zeros((0, 0), np.int16), 0)
    assert r["stats"]["phases"] == 0 and len(r["mate_b"]) == 0


def test_eviction_chain_by_hand():
    """A 2x2 case worked by hand. k = [[0, 0], [0, 5]], T = 0, diagonal scan.
    Phase 1: b0 scans a0 (admissible, k+1 = 1 = 0 + 1); b1 scans a1 (k = 5,
    no), then a0: both propose a0, b0 wins; b1 exhausts, y(b1) = 2; y(a0) = -1.
    Phase 2: B' = {b1}: a1 needs k + 1 = 6 = 0 + 2 (no); a0 needs
    k + 1 = 1 = -1 + 2 (yes): b1 takes a0 and evicts b0; y(a0) = -2.
    Phase 3: B' = {b0}, y(b0) = 1: a0 needs 1 = -2 + 1 (no), a1 needs
    1 = 0 + 1 (yes, k = 0): b0 takes a1. Done in 3 phases."""
    k = np.array([[0, 0], [0, 5]], np.int16)
    r = oracle.solve_rounded(k, 0, origin="diag")
    assert r["stats"]["phases"] == 3
    assert r["mate_b"].tolist() == [1, 0]
    assert r["y_a"].tolist() == [-2, -1] and r["y_b"].tolist() == [1, 2]
    # Each phase of a 2x2 instance with these rules is forced, so the zero
    # origin must agree here too.
    rz = oracle.solve_rounded(k, 0, origin="zero")
    assert rz["mate_b"].tolist() == [1, 0]


# ---------------------------------------- second transcription, determinism

@pytest.mark.parametrize("origin", ["diag", "zero"])
@pytest.mark.parametrize("seed", range(12))
def test_matches_independent_python_transcription(origin, seed):
    rng = np.random.default_rng(500 + seed)
    n = int(rng.integers(1, 40))
    K = int(rng.integers(0, 15))
    k = synth.random_k(n, K, seed=seed)
    T = int(rng.integers(0, max(1, n // 3)))
    r = oracle.solve_rounded(k, T, origin=origin)
    mb, ya, yb, ph, rd = tiny.solve(k.tolist(), T, origin)
    assert r["mate_b"].tolist() == mb
    assert r["y_a"].tolist() == ya and r["y_b"].tolist() == yb
    assert r["stats"]["phases"] == ph and r["stats"]["rounds"] == rd


def test_deterministic():
    k = synth.random_k(120, 20, seed=9)
    r1 = oracle.solve_rounded(k, 3, trace=True)
    r2 = oracle.solve_rounded(k, 3, trace=True)
    for x in ("mate_b", "y_a", "y_b", "trace"):
        assert np.array_equal(r1[x], r2[x])
    assert r1["stats"] == r2["stats"]


# ------------------------------------------------------- matching-based loss

def _exact_ot(X, Y):
    """min over permutations of (1/n) sum ||x_b - y_sigma(b)||^2, brute force."""
    import itertools
    n = X.shape[0]
    best, arg = None, None
    for perm in itertools.permutations(range(n)):
        v = sum(float(((X[b] - Y[perm[b]]) ** 2).sum()) for b in range(n)) / n
        if best is None or v < best:
            best, arg = v, perm
    return best, np.array(arg)


@pytest.mark.parametrize("seed", range(4))
def test_loss_gradient_equals_finite_differences_of_exact_ot(seed):
    """At generic points the optimal permutation is locally constant, so the
    gradient of the exact OT cost W(X, Y) equals the fixed-plan gradient; the
    oracle's formula must match central differences of W."""
    rng = np.random.default_rng(seed)
    n, d, h = 5, 2, 1e-5
    X = rng.standard_normal((n, d))
    Y = rng.standard_normal((n, d))
    w, perm = _exact_ot(X, Y)
    assert math.isclose(oracle.ot_loss(X, Y, perm), w, rel_tol=1e-12)
    dX, dY = oracle.ot_loss_grad(X, Y, perm)
    for M, G in ((X, dX), (Y, dY)):
        for idx in np.ndindex(M.shape):
            old = M[idx]
            M[idx] = old + h
            wp, _ = _exact_ot(X, Y)
            M[idx] = old - h
            wm, _ = _exact_ot(X, Y)
            M[idx] = old
            assert abs((wp - wm) / (2 * h) - G[idx]) < 1e-6


def test_loss_gradient_scales_with_upstream_gradient():
    rng = np.random.default_rng(1)
    X, Y = rng.standard_normal((6, 3)), rng.standard_normal((6, 3))
    mb = rng.permutation(6)
    a1, b1 = oracle.ot_loss_grad(X, Y, mb, 1.0)
    a3, b3 = oracle.ot_loss_grad(X, Y, mb, -3.0)
    assert np.allclose(a3, -3.0 * a1) and np.allclose(b3, -3.0 * b1)
    # the two gradients are opposite on matched pairs: sum over all is zero
    assert np.allclose(a1.sum(0) + b1.sum(0), 0.0)


def test_points_max_and_pairs_equal_full_matrix():
    """The large-instance helpers reproduce round_points_f32 exactly."""
    rng = np.random.default_rng(21)
    for n, d, eps in [(1, 2, 0.1), (37, 3, 0.01), (200, 2, 0.005), (64, 5, 0.05)]:
        X = rng.random((n, d), dtype=np.float32)
        Y = rng.random((n, d), dtype=np.float32)
        k, m = oracle.round_points_f32(X, Y, eps)
        assert oracle.points_max_f32(X, Y) == m
        b = rng.integers(0, n, 300)
        a = rng.integers(0, n, 300)
        assert np.array_equal(oracle.points_pairs_f32(X, Y, eps, m, b, a), k[b, a])
    X = np.full((5, 2), 0.5, np.float32)
    assert oracle.points_max_f32(X, X) == 0.0
    assert (oracle.points_pairs_f32(X, X, 0.1, 0.0, [0, 4], [3, 1]) == 0).all()


# ------------------------------------------- point sets without the matrix

def _grid_points(n, d, seed, top=7):
    rng = np.random.default_rng(seed)
    return rng.integers(0, top + 1, (n, d)).astype(np.float32)


@pytest.mark.parametrize("n_b,n_a,d,origin", [(40, 40, 2, "diag"), (33, 47, 3, "zero"),
                                              (60, 60, 3, "diag")])
def test_points_without_matrix_exact_grid(n_b, n_a, d, origin):
    """Integer points (every binary32 step exact) and eps = 1/8: eq. (1) is
    floor(8 d2 / m) exactly, computed here with integers. The loop that
    computes each cost from the points runs the same trajectory as the loop
    on that exact matrix, and its final state meets (I1), (I2) on the exact
    costs, Lemma 3.1 (sum_M k <= OPT_k + n_b, OPT_k by scipy's exact
    assignment) and the stop test."""
    X = _grid_points(n_b, d, seed=n_b + d)
    Y = _grid_points(n_a, d, seed=n_a + 7 * d)
    d2 = ((X.astype(np.int64)[:, None, :] - Y.astype(np.int64)[None, :, :]) ** 2).sum(-1)
    m = int(d2.max())
    k = (8 * d2) // m
    eps = 0.125
    T = oracle.threshold(eps, n_b)
    r = oracle.solve_points(X, Y, eps, origin=origin, complete=False, trace=True)
    assert r["m"] == m
    ref = oracle.solve_rounded(k.astype(np.int16), T, origin=origin, complete=False, trace=True)
    for x in ("mate_a", "mate_b", "y_a", "y_b", "trace"):
        assert np.array_equal(r[x], ref[x]), x
    assert r["stats"] == ref["stats"]
    check_matching(r["mate_a"], r["mate_b"])
    check_I1(r["mate_a"], r["y_a"], r["y_b"])
    check_I2(k, r["mate_b"], r["y_a"], r["y_b"])
    assert (r["mate_b"] < 0).sum() <= T
    rows, cols = linear_sum_assignment(k)
    opt = int(k[rows, cols].sum())
    mb = r["mate_b"]
    got = int(k[np.nonzero(mb >= 0)[0], mb[mb >= 0]].sum())
    assert got <= opt + n_b


@pytest.mark.parametrize("n_b,n_a,d,eps", [(300, 300, 2, 0.05), (257, 311, 3, 0.01),
                                           (120, 150, 16, 0.05)])
def test_points_without_matrix_equals_the_rounded_matrix(n_b, n_a, d, eps):
    """On generic (non-grid) points the loop that computes each cost from
    the points gives what the loop gives on round_points_f32's matrix (itself
    pinned by exact rationals above): mates, duals, statistics and trace."""
    rng = np.random.default_rng(n_b * d)
    X = rng.random((n_b, d), dtype=np.float32)
    Y = (rng.random((n_a, d), dtype=np.float32) * 1.5).astype(np.float32)
    k, m = oracle.round_points_f32(X, Y, eps)
    for origin in ("diag", "zero"):
        a = oracle.solve_rounded(k, oracle.threshold(eps, n_b), origin=origin, trace=True)
        b = oracle.solve_points(X, Y, eps, origin=origin, trace=True)
        for x in ("mate_a", "mate_b", "y_a", "y_b", "trace"):
            assert np.array_equal(a[x], b[x]), (origin, x)
        assert a["stats"] == b["stats"] and b["m"] == m


# ---------------------------------------------------------------- unbalanced

def _rect_case(n_b, n_a, K, seed):
    rng = np.random.default_rng(seed)
    return rng.integers(0, K + 1, (n_b, n_a)).astype(np.int16)


@pytest.mark.parametrize("origin", ["diag", "zero"])
@pytest.mark.parametrize("n_b,n_a,K,T", [(5, 9, 6, 0), (20, 31, 8, 1), (40, 41, 10, 2),
                                         (1, 7, 5, 0), (33, 100, 12, 3)])
def test_unbalanced_phase_invariants(n_b, n_a, K, T, origin):
    """|B| < |A| (Section 3.3): every phase keeps (I1), (I2), Lemma 2.1,
    a maximal admissible M', the step (III) updates and Lemma 3.3 exactly; the
    loop ends with |B'| <= T, within the phase bound of Lemma 3.2 over all
    n_b + n_a vertices."""
    k = _rect_case(n_b, n_a, K, seed=n_b * 7 + n_a)
    state = None
    phases = sum_free = 0
    while True:
        r = oracle.solve_rounded(k, T, origin=origin, max_phases=1, state=state, complete=False)
        before = state if state is not None else dict(
            mate_a=np.full(n_a, -1), mate_b=np.full(n_b, -1), y_a=np.zeros(n_a, np.int64),
            y_b=np.ones(n_b, np.int64))
        if r["stats"]["phases"] == 0:
            break
        check_matching(r["mate_a"], r["mate_b"])
        check_I1(r["mate_a"], r["y_a"], r["y_b"])
        check_I2(k, r["mate_b"], r["y_a"], r["y_b"])
        sum_free += check_phase(k, before, r)
        phases += 1
        state = r
    final = state if state is not None else oracle.solve_rounded(k, T, origin=origin, complete=False)
    assert (np.asarray(final["mate_b"]) < 0).sum() <= T
    full = oracle.solve_rounded(k, T, origin=origin, complete=False)
    assert full["stats"]["phases"] == phases and full["stats"]["sum_free"] == sum_free
    for key in ("mate_a", "mate_b", "y_a", "y_b"):
        assert np.array_equal(full[key], final[key])
    bound_free, bound_phases = safe_phase_bounds(n_b, K, T, n_a)
    assert sum_free <= bound_free and phases <= bound_phases


@pytest.mark.parametrize("n_b,n_a,eps", [(30, 45, 0.1), (60, 61, 0.05), (25, 200, 0.02),
                                         (100, 150, 0.05)])
def test_unbalanced_lemma_3_5_and_total_error(n_b, n_a, eps):
    """Lemma 3.5: the loop's matching (size >= (1 - eps)|B|) costs at most
    eps |B| more than an optimal |B|-matching under the rounded costs, i.e.
    sum_M k <= OPT_k + |B|; after the completion the true cost is within
    3 eps |B| of the optimal |B|-matching."""
    rng = np.random.default_rng(n_b + n_a)
    C = rng.random((n_b, n_a), dtype=np.float32)
    C[0, 0] = 1.0
    k = oracle.round_cost(C, eps)
    T = oracle.threshold(eps, n_b)
    r = oracle.solve_rounded(k, T, complete=False)
    mb = np.asarray(r["mate_b"])
    matched = np.nonzero(mb >= 0)[0]
    assert len(matched) >= n_b - T
    rows, cols = linear_sum_assignment(k.astype(np.int64))
    opt_k = int(k.astype(np.int64)[rows, cols].sum())
    assert int(k.astype(np.int64)[matched, mb[matched]].sum()) <= opt_k + n_b
    done = oracle.solve_rounded(k, T)
    mb = np.asarray(done["mate_b"])
    assert (mb >= 0).all()
    check_matching(done["mate_a"], mb)
    c64 = C.astype(np.float64)
    rows, cols = linear_sum_assignment(c64)
    opt = c64[rows, cols].sum()
    assert c64[np.arange(n_b), mb].sum() <= opt + 3 * eps * n_b + 1e-9


def test_unbalanced_closed_forms():
    """One row: its dual rises one step per phase until its smallest cost is
    admissible, so there are min k + 1 phases and it takes the first column
    of smallest cost in its scan order; T >= |B| runs no phase and the
    completion pairs rows with the lowest free columns."""
    k = np.array([[5, 3, 7, 3, 9]], np.int16)
    for origin, want in (("diag", 1), ("zero", 1)):
        r = oracle.solve_rounded(k, 0, origin=origin)
        assert r["stats"]["phases"] == 4 and r["mate_b"][0] == want
        assert r["y_b"][0] == 4 and r["y_a"][want] == -1
    k = _rect_case(4, 6, 3, seed=1)
    r = oracle.solve_rounded(k, 4)
    assert r["stats"]["phases"] == 0
    assert list(r["mate_b"]) == [0, 1, 2, 3] and list(r["mate_a"]) == [0, 1, 2, 3, -1, -1]
