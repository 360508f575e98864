"""Pins of the oracle's clustered transport (Section 4 with Lemma 4.1): the
copies of every point kept as a top dual, a free count and pair counts by
the parity of the demand copy's level.

Checked against: the assignment loop (one copy per point is exactly the
Section 2.2 loop, matchings, duals and statistics); an independent Python
run of the same reading on explicit copies that assumes nothing from Lemma
4.1 (`tiny.solve_point_rounds_on_copies`), phase by phase; after every
phase, on the copies the clusters stand for: (I1), (I2), Lemma 4.1, the
free-copy raise, and that the phase's M' is admissible, within the
capacities and maximal; exact transport LPs (cost <= OPT + 3.5 eps) and
forced plans."""
import math

import numpy as np
import pytest

import oracle
from oracle import tiny

scipy_opt = pytest.importorskip("scipy.optimize")


def _masses(rng, n, zeros=0):
    w = rng.random(n) + 0.05
    if zeros:
        w[rng.choice(n, zeros, replace=False)] = 0.0
    return w / w.sum()


def _exact_ot(C, nu, mu):
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


def _instance(rng, n_b, n_a, eps, zeros=0):
    C = rng.random((n_b, n_a)).astype(np.float32)
    nu, mu = _masses(rng, n_b, zeros), _masses(rng, n_a)
    s, d, _ = oracle.ot_scale(nu, mu, eps)
    k = oracle.round_cost(C, eps)
    T = int(math.floor(eps * int(s.sum()) + 1e-9))
    return C, nu, mu, s, d, k, T


@pytest.mark.parametrize("origin", ["diag", "zero"])
def test_one_copy_per_point_is_the_assignment_loop(origin):
    """With s = d = 1 every cluster is a single copy and the point-level
    rounds are the copy-level rounds of Section 2.2."""
    rng = np.random.default_rng(7)
    for it in range(60):
        n_b = int(rng.integers(1, 30))
        n_a = int(rng.integers(n_b, 36))
        k = rng.integers(0, int(rng.integers(1, 12)), (n_b, n_a)).astype(np.int16)
        T = int(rng.integers(0, 3))
        r = oracle.ot_clustered_rounded(k, np.ones(n_b), np.ones(n_a), T, origin)
        a = oracle.solve_rounded(k, T, origin)
        assert r["status"] == "ok"
        mate_b = np.array([int(np.argmax(row)) if row.any() else -1 for row in r["flow"]])
        assert (r["flow"].sum(1) == 1).all() and (r["flow"].sum(0) <= 1).all()
        assert np.array_equal(mate_b, a["mate_b"]), it
        assert np.array_equal(r["Y"], a["y_b"]) and np.array_equal(r["Z"], a["y_a"]), it
        assert r["stats"] == a["stats"], it


@pytest.mark.parametrize("origin", ["diag", "zero"])
@pytest.mark.parametrize("n_b,n_a,eps,seed", [(3, 4, 0.25, 0), (4, 4, 0.2, 1), (5, 3, 0.25, 2),
                                              (2, 6, 0.2, 3), (6, 2, 0.3, 4), (1, 5, 0.2, 5),
                                              (5, 1, 0.2, 6)])
def test_matches_copy_level_run_phase_by_phase(n_b, n_a, eps, seed, origin):
    rng = np.random.default_rng(seed)
    C, nu, mu, s, d, k, T = _instance(rng, n_b, n_a, eps)
    snaps, flow, phases, rounds = tiny.solve_point_rounds_on_copies(
        k.tolist(), s.tolist(), d.tolist(), T, origin)
    state = None
    for t, (Y, F, Z, G, w) in enumerate(snaps):
        r = oracle.ot_clustered_rounded(k, s, d, T, origin, max_phases=1, state=state,
                                        complete=False)
        assert r["stats"]["phases"] == 1
        assert r["Y"].tolist() == Y and r["F"].tolist() == F, f"phase {t + 1}"
        assert r["Z"].tolist() == Z and r["G"].tolist() == G, f"phase {t + 1}"
        assert r["w"].tolist() == w, f"phase {t + 1}"
        state = {x: r[x] for x in ("Y", "F", "Z", "G", "w")}
    full = oracle.ot_clustered_rounded(k, s, d, T, origin)
    assert full["flow"].tolist() == flow
    assert full["stats"]["phases"] == phases and full["stats"]["rounds"] == rounds


def _copy_levels(k, st):
    """The duals of the copies the clusters stand for, per point: supply
    point b -> {level: count}, demand point a -> {level: count}."""
    k = np.asarray(k, np.int64)
    Y, F, Z, G, w = (np.asarray(st[x]) for x in ("Y", "F", "Z", "G", "w"))
    n_b, n_a = k.shape
    sup = [{} for _ in range(n_b)]
    dem = [{} for _ in range(n_a)]
    for b in range(n_b):
        if F[b]:
            sup[b][int(Y[b])] = sup[b].get(int(Y[b]), 0) + int(F[b])
    for a in range(n_a):
        if G[a]:
            dem[a][0] = dem[a].get(0, 0) + int(G[a])
    for b in range(n_b):
        for a in range(n_a):
            for p in (0, 1):
                c = int(w[b, a, p])
                if not c:
                    continue
                za = int(Z[a]) if (int(Z[a]) & 1) == p else int(Z[a]) - 1
                yb = int(k[b, a]) - za  # the pair is tight
                sup[b][yb] = sup[b].get(yb, 0) + c
                dem[a][za] = dem[a].get(za, 0) + c
    return sup, dem


@pytest.mark.parametrize("origin", ["diag", "zero"])
@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_copies_after_every_phase(seed, origin):
    """After every phase, on the copies: each point's copies hold at most two
    duals, one apart (Lemma 4.1), with the free supply copies at the largest
    (the raise) and the free demand copies at 0; the tops are what the state
    says; (I1) y(b) >= 0 >= y(a); eq. (2) on every pair of copies (enough:
    top + top <= k + 1); counts conserved; the phase's M' uses admissible
    edges only, within the free copies and the demand points' top copies, and
    is maximal; sum F never grows, Y never falls, Z never rises."""
    rng = np.random.default_rng(40 + seed)
    n_b, n_a, eps = 7, 6, 0.1
    C, nu, mu, s, d, k, T = _instance(rng, n_b, n_a, eps, zeros=1)
    k64 = k.astype(np.int64)
    prev = None
    while True:
        r = oracle.ot_clustered_rounded(k, s, d, T, origin, max_phases=1, state=prev,
                                        complete=False, want_last=True)
        if r["stats"]["phases"] == 0:
            break
        st = {x: r[x] for x in ("Y", "F", "Z", "G", "w")}
        sup, dem = _copy_levels(k, st)
        for b in range(n_b):
            assert sum(sup[b].values()) == s[b]
            if s[b]:
                assert max(sup[b]) == st["Y"][b] and max(sup[b]) - min(sup[b]) <= 1
                assert min(sup[b]) >= 1
        for a in range(n_a):
            assert sum(dem[a].values()) == d[a]
            if d[a]:
                assert max(dem[a]) == st["Z"][a] and max(dem[a]) - min(dem[a]) <= 1
                assert max(dem[a]) <= 0
            if st["G"][a]:
                assert st["Z"][a] == 0
        assert (st["Y"][:, None].astype(np.int64) + st["Z"][None, :] <= k64 + 1).all()
        # M' against the state it started from
        p0 = prev if prev is not None else {
            "Y": np.ones(n_b, np.int32), "F": s.astype(np.int64), "Z": np.zeros(n_a, np.int32),
            "G": d.astype(np.int64), "w": np.zeros((n_b, n_a, 2), np.int64)}
        _, dem0 = _copy_levels(k, p0)
        top0 = np.array([dem0[a].get(int(p0["Z"][a]), 0) for a in range(n_a)])
        adm = (p0["Y"][:, None].astype(np.int64) + p0["Z"][None, :] == k64 + 1)
        adm &= (np.asarray(p0["F"]) > 0)[:, None]
        m = r["m_last"]
        assert (m[~adm] == 0).all(), "M' uses an edge that is not admissible"
        assert (m.sum(1) <= p0["F"]).all() and (m.sum(0) <= top0).all()
        short = m.sum(1) < p0["F"]
        full_a = m.sum(0) == top0
        assert not (adm[short] & ~full_a[None, :] & (top0 > 0)[None, :]).any(), "M' not maximal"
        assert st["F"].sum() <= np.asarray(p0["F"]).sum()
        assert (st["Y"] >= p0["Y"]).all() and (st["Z"] <= p0["Z"]).all()
        prev = st


@pytest.mark.parametrize("origin", ["diag", "zero"])
@pytest.mark.parametrize("n_b,n_a,eps,seed", [(4, 5, 0.1, 0), (6, 6, 0.1, 1), (8, 5, 0.2, 2),
                                              (5, 8, 0.05, 3), (3, 3, 0.02, 4)])
def test_plan_feasible_and_within_bound_of_exact_ot(n_b, n_a, eps, seed, origin):
    rng = np.random.default_rng(seed)
    C = rng.random((n_b, n_a)).astype(np.float32)
    nu, mu = _masses(rng, n_b), _masses(rng, n_a)
    r = oracle.ot_solve_clustered(C, nu, mu, eps, origin=origin)
    P = r["plan"]
    assert r["status"] == "ok" and (P >= 0).all()
    assert np.allclose(P.sum(1), nu, rtol=0, atol=1e-12)
    assert (P.sum(0) <= mu + 1e-12).all()
    assert math.isclose(r["cost"], float((P * C.astype(np.float64)).sum()), rel_tol=1e-12,
                        abs_tol=1e-15)
    assert r["repaired"] <= eps / 2 + 1e-12
    opt = _exact_ot(C, nu, mu)
    assert opt - 1e-9 <= r["cost"] <= opt + 3.5 * eps


def test_forced_plans():
    rng = np.random.default_rng(3)
    C = rng.random((1, 6)).astype(np.float32)
    mu = _masses(rng, 6)
    r = oracle.ot_solve_clustered(C, np.ones(1), mu, 0.1)
    assert np.allclose(r["plan"][0], mu, rtol=0, atol=1e-12)
    C = rng.random((5, 1)).astype(np.float32)
    nu = _masses(rng, 5)
    r = oracle.ot_solve_clustered(C, nu, np.ones(1), 0.1)
    assert np.allclose(r["plan"][:, 0], nu, rtol=0, atol=1e-12)


def test_cluster_counts_and_levels():
    """Copies per level from the state: supply copies at Y_b and Y_b - 1 sum
    to s_b, demand copies at Z_a and Z_a - 1 to d_a."""
    rng = np.random.default_rng(9)
    C = rng.random((9, 7)).astype(np.float32)
    nu, mu = _masses(rng, 9, zeros=2), _masses(rng, 7)
    r = oracle.ot_solve_clustered(C, nu, mu, 0.05)
    assert np.array_equal(r["b_hi"] + r["b_lo"], r["s"])
    assert np.array_equal(r["a_top"] + r["a_bot"], r["d"])
    assert r["stats"]["completed_pairs"] == int(r["F"].sum())


def test_more_supply_points_than_demand_points():
    """The scan of supply point b starts at column b mod n_a."""
    rng = np.random.default_rng(11)
    C = rng.random((12, 3)).astype(np.float32)
    nu, mu = _masses(rng, 12), _masses(rng, 3)
    for origin in ("diag", "zero"):
        r = oracle.ot_solve_clustered(C, nu, mu, 0.05, origin=origin)
        opt = _exact_ot(C, nu, mu)
        assert r["status"] == "ok" and opt - 1e-9 <= r["cost"] <= opt + 3.5 * 0.05


def test_transport_clouds_eps_001_n1000_runs():
    """The size the clusters are for: theta = 400,000 copies a side."""
    from paper_2203_03732_amd import synth
    C, nu, mu = synth.transport_clouds(1000, 1000, seed=11, shift=1)
    r = oracle.ot_solve_clustered(C, nu, mu, 0.01)
    assert r["status"] == "ok"
    P = r["plan"]
    assert np.allclose(P.sum(1), nu, rtol=0, atol=1e-12) and (P.sum(0) <= mu + 1e-12).all()
    assert r["s"].sum() > 390000 and r["stats"]["phases"] > 100
    assert np.array_equal(r["b_hi"] + r["b_lo"], r["s"])
