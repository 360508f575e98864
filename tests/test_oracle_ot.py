"""Pins of the oracle's optimal-transport reduction (Section 4): scaling of
the masses, the copies' phase loop with the free-copy dual raise, and the
plan after the feasibility repair. Checked against exact linear programs
(scipy's HiGHS), forced plans, hand-computed scalings, Lemma 4.1 and the
invariants of Section 2 after every phase, and an independent Python
transcription of the copies' loop."""
import math

import numpy as np
import pytest

import oracle
from oracle import tiny
from invariants import check_I1, check_I2

scipy_opt = pytest.importorskip("scipy.optimize")


def _masses(rng, n, zeros=0):
    w = rng.random(n) + 0.05
    if zeros:
        w[rng.choice(n, zeros, replace=False)] = 0.0
    return w / w.sum()


def _exact_ot(C, nu, mu):
    """Optimal transport cost by linear programming (equality on both sides)."""
    n_b, n_a = C.shape
    A = []
    for b in range(n_b):
        row = np.zeros((n_b, n_a))
        row[b, :] = 1
        A.append(row.ravel())
    for a in range(n_a):
        col = np.zeros((n_b, n_a))
        col[:, a] = 1
        A.append(col.ravel())
    res = scipy_opt.linprog(np.asarray(C, np.float64).ravel(), A_eq=np.array(A),
                            b_eq=np.concatenate([nu, mu]), bounds=(0, None), method="highs")
    assert res.status == 0
    return float(res.fun)


def test_scale_hand_values():
    s, d, th = oracle.ot_scale([0.5, 0.25, 0.25], [0.5, 0.5], 0.1)
    assert th == 120.0
    assert s.tolist() == [60, 30, 30] and d.tolist() == [60, 60]
    # 0.7 * 48 = 33.6 (down: 33), 0.3 * 48 = 14.4 (14); 0.2 * 48 = 9.6 (up: 10),
    # 14.4 (15), 0.5 * 48 = 24 exactly (24)
    s, d, th = oracle.ot_scale([0.7, 0.3], [0.2, 0.3, 0.5], 0.25)
    assert th == 48.0
    assert s.tolist() == [33, 14] and d.tolist() == [10, 15, 24]


def test_scale_rejects_bad_masses():
    with pytest.raises(oracle.OracleError, match="range"):
        oracle.ot_scale([0.5, 0.4], [0.5, 0.5], 0.1)
    with pytest.raises(oracle.OracleError, match="range"):
        oracle.ot_scale([1.5, -0.5], [0.5, 0.5], 0.1)
    with pytest.raises(oracle.OracleError, match="range"):
        oracle.ot_scale([float("nan"), 1.0], [0.5, 0.5], 0.1)
    with pytest.raises(oracle.OracleError, match="eps"):
        oracle.ot_scale([1.0], [1.0], 0.0)


def _check_plan(r, C, nu, mu, eps):
    P = r["plan"]
    assert P is not None and r["status"] == "ok"
    assert (P >= 0).all()
    assert np.allclose(P.sum(1), nu, rtol=0, atol=1e-12), "a supply point is not fully sent"
    assert (P.sum(0) <= mu + 1e-12).all(), "a demand point receives more than its mass"
    want = float((P * np.asarray(C, np.float64)).sum())
    assert math.isclose(r["cost"], want, rel_tol=1e-12, abs_tol=1e-15)
    # the repair moves at most (n_b + n_a) / theta <= eps / 2
    assert r["repaired"] <= (len(nu) + len(mu)) / r["theta"] + 1e-12
    assert r["repaired"] <= eps / 2 + 1e-12


def test_single_supply_point_forced_plan():
    """With one supply point every feasible plan sends mu_a to each a."""
    rng = np.random.default_rng(1)
    C = rng.random((1, 9)).astype(np.float32)
    mu = _masses(rng, 9, zeros=2)
    r = oracle.ot_solve(C, [1.0], mu, 0.1)
    _check_plan(r, C, np.array([1.0]), mu, 0.1)
    assert np.allclose(r["plan"][0], mu, rtol=0, atol=1e-12)


def test_single_demand_point_forced_plan():
    rng = np.random.default_rng(2)
    C = rng.random((7, 1)).astype(np.float32)
    nu = _masses(rng, 7)
    r = oracle.ot_solve(C, nu, [1.0], 0.2)
    _check_plan(r, C, nu, np.array([1.0]), 0.2)
    assert np.allclose(r["plan"][:, 0], nu, rtol=0, atol=1e-12)


@pytest.mark.parametrize("origin", ["diag", "zero"])
@pytest.mark.parametrize("n_b,n_a,eps,seed", [(3, 3, 0.2, 0), (5, 8, 0.1, 1), (9, 4, 0.1, 2),
                                              (12, 12, 0.05, 3), (6, 10, 0.25, 4),
                                              (15, 11, 0.1, 5)])
def test_plan_feasible_and_within_bound_of_exact_ot(n_b, n_a, eps, seed, origin):
    """cost <= OPT + 3 eps (the copies' matching: Lemma 3.5 plus rounding and
    completion, per unit of the at most theta copies) + eps / 2 (the repair,
    each unit of moved mass costing at most 1)."""
    rng = np.random.default_rng(seed)
    C = rng.random((n_b, n_a)).astype(np.float32)
    C[0, 0] = 1.0
    nu = _masses(rng, n_b, zeros=1 if n_b > 4 else 0)
    mu = _masses(rng, n_a)
    r = oracle.ot_solve(C, nu, mu, eps, origin=origin)
    _check_plan(r, C, nu, mu, eps)
    opt = _exact_ot(C, nu, mu)
    assert r["cost"] <= opt + 3.5 * eps + 1e-9
    assert r["cost"] >= opt - 1e-9
    s, d, th = oracle.ot_scale(nu, mu, eps)
    assert len(r["mate_b"]) == s.sum() and len(r["mate_a"]) == d.sum()
    assert r["T"] == oracle.threshold(eps, int(s.sum()))


def test_equal_masses_reduce_to_assignment():
    """nu = mu = 1/n: the exact transport cost is the optimal assignment / n
    (Birkhoff), here from scipy's assignment solver."""
    from scipy.optimize import linear_sum_assignment
    rng = np.random.default_rng(7)
    n, eps = 10, 0.05
    C = rng.random((n, n)).astype(np.float32)
    r = oracle.ot_solve(C, np.full(n, 1 / n), np.full(n, 1 / n), eps)
    rows, cols = linear_sum_assignment(C.astype(np.float64))
    opt = float(C.astype(np.float64)[rows, cols].sum()) / n
    _check_plan(r, C, np.full(n, 1 / n), np.full(n, 1 / n), eps)
    assert opt - 1e-12 <= r["cost"] <= opt + 3.5 * eps


def _copy_k(C, r, eps):
    kp = oracle.round_cost(C, eps).astype(np.int64)
    ob = np.repeat(np.arange(len(r["s"])), r["s"])
    oa = np.repeat(np.arange(len(r["d"])), r["d"])
    return kp[np.ix_(ob, oa)], ob, oa


@pytest.mark.parametrize("origin", ["diag", "zero"])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_two_clusters_and_raise_after_every_phase(seed, origin):
    """After every phase: each supply point's free copies hold the largest
    dual of its copies, and the copies of every point (supply or demand) hold
    at most two dual values, one apart (Lemma 4.1); (I1), (I2) on the copies;
    duals of supply copies never fall, of demand copies never rise; a matched
    demand copy stays matched (Lemma 2.1). Resuming phase by phase gives the
    one-shot result."""
    rng = np.random.default_rng(100 + seed)
    n_b, n_a, eps = 6, 7, 0.2
    C = rng.random((n_b, n_a)).astype(np.float32)
    nu, mu = _masses(rng, n_b), _masses(rng, n_a)
    full = oracle.ot_solve(C, nu, mu, eps, origin=origin)
    k, ob, oa = _copy_k(C, full, eps)
    state, phases = None, 0
    while True:
        r = oracle.ot_solve(C, nu, mu, eps, origin=origin, max_phases=1, state=state)
        phases += r["stats"]["phases"]
        if r["status"] == "ok":  # the stop test held (after at most one phase)
            break
        mb, ma, yb, ya = r["mate_b"], r["mate_a"], r["y_b"], r["y_a"]
        check_I1(ma, ya, yb)
        check_I2(k, mb, ya, yb)
        for p in range(n_b):
            v = yb[ob == p]
            if len(v):
                assert v.max() - v.min() <= 1, f"phase {phases}: supply point {p} duals {set(v)}"
                assert (v[mb[ob == p] < 0] == v.max()).all(), "a free copy was not raised"
        for q in range(n_a):
            v = ya[oa == q]
            if len(v):
                assert v.max() - v.min() <= 1, f"phase {phases}: demand point {q} duals {set(v)}"
        if state is not None:
            assert (yb >= state["y_b"]).all() and (ya <= state["y_a"]).all()
            assert (ma[state["mate_a"] >= 0] >= 0).all()
        state = {x: r[x] for x in ("mate_a", "mate_b", "y_a", "y_b")}
    assert phases == full["stats"]["phases"]
    for x in ("mate_a", "mate_b", "y_a", "y_b"):
        assert np.array_equal(r[x], full[x])
    assert np.array_equal(r["plan"], full["plan"])


@pytest.mark.parametrize("origin", ["diag", "zero"])
@pytest.mark.parametrize("n_b,n_a,eps,seed", [(3, 4, 0.25, 0), (4, 4, 0.2, 1), (5, 3, 0.25, 2),
                                              (2, 6, 0.2, 3)])
def test_copies_match_independent_transcription(n_b, n_a, eps, seed, origin):
    rng = np.random.default_rng(seed)
    C = rng.random((n_b, n_a)).astype(np.float32)
    nu, mu = _masses(rng, n_b), _masses(rng, n_a)
    r = oracle.ot_solve(C, nu, mu, eps, origin=origin)
    kp = oracle.round_cost(C, eps).tolist()
    mb, ya, yb, ph, rd = tiny.solve_copies(kp, r["s"].tolist(), r["d"].tolist(), r["T"], origin)
    assert mb == r["mate_b"].tolist()
    assert ya == r["y_a"].tolist() and yb == r["y_b"].tolist()
    assert ph == r["stats"]["phases"] and rd == r["stats"]["rounds"]
