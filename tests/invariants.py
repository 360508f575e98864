"""Checks of what arXiv:2203.03732 proves about the phase loop.

Independent numpy code used by the tests against both the CPU oracle and the
GPU library. Units: rounded costs k and duals y in integer steps of eps;
k[b, a] with rows = supply B and columns = demand A.
"""
from __future__ import annotations

import itertools

import numpy as np


def check_matching(mate_a, mate_b, perfect=False):
    n_b, n_a = len(mate_b), len(mate_a)
    mb = np.asarray(mate_b)
    ma = np.asarray(mate_a)
    for b in range(n_b):
        a = mb[b]
        if a >= 0:
            assert 0 <= a < n_a and ma[a] == b, f"mate arrays disagree at b={b}"
    for a in range(n_a):
        b = ma[a]
        if b >= 0:
            assert 0 <= b < n_b and mb[b] == a, f"mate arrays disagree at a={a}"
    if perfect:
        assert (mb >= 0).all(), "matching is not perfect"


def mate_a_from_mate_b(mate_b, n_a):
    ma = np.full(n_a, -1, np.int64)
    for b, a in enumerate(np.asarray(mate_b)):
        if a >= 0:
            assert ma[a] < 0, "two b share one a"
            ma[a] = b
    return ma


def check_I1(mate_a, y_a, y_b):
    """(I1): y(b) >= 0, y(a) <= 0, and every free a has y(a) = 0."""
    y_a = np.asarray(y_a)
    y_b = np.asarray(y_b)
    assert (y_b >= 0).all(), "a supply dual went negative"
    assert (y_a <= 0).all(), "a demand dual went positive"
    free_a = np.asarray(mate_a) < 0
    assert (y_a[free_a] == 0).all(), "a free demand vertex has a nonzero dual"


def check_I2(k, mate_b, y_a, y_b):
    """(I2), eqs. (2)-(3): y(a)+y(b) <= k+1 off M and y(a)+y(b) = k on M."""
    k = np.asarray(k, dtype=np.int64)
    S = np.asarray(y_b, np.int64)[:, None] + np.asarray(y_a, np.int64)[None, :]
    assert (S <= k + 1).all(), "eq. (2) violated"
    mb = np.asarray(mate_b)
    bs = np.nonzero(mb >= 0)[0]
    if len(bs):
        assert (S[bs, mb[bs]] == k[bs, mb[bs]]).all(), "eq. (3) violated"


def potential(y_a, y_b):
    """Phi = sum |y| = sum y(b) - sum y(a) (signs fixed by (I1))."""
    return int(np.sum(np.asarray(y_b, np.int64)) - np.sum(np.asarray(y_a, np.int64)))


def check_phase(k, before, after):
    """One phase, from the state `before` to the state `after`.

    Checks Lemma 2.1, that M' holds only admissible edges and is maximal in
    the admissible graph of B', the dual update rules of step (III), and the
    exact form of Lemma 3.3 (Phi grows by exactly |B'|). Returns |B'|."""
    k = np.asarray(k, dtype=np.int64)
    mb0, ma0 = np.asarray(before["mate_b"]), np.asarray(before["mate_a"])
    mb1, ma1 = np.asarray(after["mate_b"]), np.asarray(after["mate_a"])
    ya0, yb0 = np.asarray(before["y_a"], np.int64), np.asarray(before["y_b"], np.int64)
    ya1, yb1 = np.asarray(after["y_a"], np.int64), np.asarray(after["y_b"], np.int64)
    F = np.nonzero(mb0 < 0)[0]
    # Lemma 2.1: every a matched before stays matched.
    assert (ma1[ma0 >= 0] >= 0).all(), "a matched demand vertex became free"
    # M' = new edges, all incident on B'.
    new_b = np.nonzero((mb1 >= 0) & (mb1 != mb0))[0]
    assert np.isin(new_b, F).all(), "a vertex outside B' changed partner"
    won = np.zeros(len(mb0), bool)
    won[new_b] = True
    taken = np.zeros(len(ma0), bool)
    taken[mb1[new_b]] = True
    admissible = (k + 1) == (yb0[:, None] + ya0[None, :])
    assert admissible[new_b, mb1[new_b]].all(), "M' holds a non-admissible edge"
    # Maximality: no admissible edge joins a b of B' left free and an untaken a.
    lost = F[~won[F]]
    if len(lost):
        assert not (admissible[lost][:, ~taken]).any(), "M' is not maximal"
    # Step (III): y(a) -= 1 exactly on M' columns; y(b) += 1 exactly on lost.
    assert np.array_equal(ya1, ya0 - taken.astype(np.int64)), "y(a) update wrong"
    inc = np.zeros(len(mb0), np.int64)
    inc[lost] = 1
    assert np.array_equal(yb1, yb0 + inc), "y(b) update wrong"
    # Lemma 3.3, exact: each b in B' adds one unit to |y| somewhere.
    assert potential(ya1, yb1) - potential(ya0, yb0) == len(F)
    return len(F)


def safe_phase_bounds(n, K, T, n_a=None):
    """Bounds on sum |B'| and on the phase count from Lemma 3.2 applied to all
    n_b + n_a vertices: Phi <= (n_b + n_a)(K+2), Phi starts at n_b, each phase
    adds n_i > T. (n_b = n; n_a = n unless given.)"""
    n_a = n if n_a is None else n_a
    sum_free = (n + n_a) * (K + 2) - n
    return sum_free, sum_free // (T + 1)


def brute_force_opt(c):
    """Minimum over all perfect matchings of sum c[b, perm[b]] (n <= 8)."""
    c = np.asarray(c, dtype=np.float64)
    n = c.shape[0]
    best = None
    rows = np.arange(n)
    for perm in itertools.permutations(range(n)):
        v = c[rows, list(perm)].sum()
        if best is None or v < best:
            best = v
    return 0.0 if best is None else best


def matching_cost(c, mate_b):
    c = np.asarray(c, dtype=np.float64)
    mb = np.asarray(mate_b)
    return float(c[np.arange(len(mb)), mb].sum())
