"""Pins of the oracle's cost variants of Section 5: the plain Euclidean
distance (the synthetic experiment) and half the L1 distance of vectors
normalised to sum 1 (the image experiment). Checked against exact rational
arithmetic on inputs where the binary32 steps are exact, hand-worked values,
binary64 references (differences only next to rounding boundaries),
invariances and rejections."""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_2203_03732_amd import synth


def _exact_floor_sqrt_ratio(d2: int, m: int, eps: float):
    """floor(sqrt(d2/m) / eps) in exact arithmetic, and whether sqrt(d2/m)/eps
    lies within 1e-9 of an integer (where binary64 rounding may decide)."""
    e = Fraction(eps)
    r = Fraction(d2, m)
    x = math.sqrt(d2 / m) / eps
    j = int(math.floor(x)) + 1
    while j > 0 and (j * e) ** 2 > r:
        j -= 1
    while ((j + 1) * e) ** 2 <= r:
        j += 1
    return j, abs(x - round(x)) < 1e-9


def test_euclid_hand_values():
    X = np.array([[0.0, 0.0]], np.float32)
    Y = np.array([[3.0, 4.0], [0.0, 5.0], [6.0, 8.0], [0.0, 0.0]], np.float32)
    k, m = oracle.round_points_euclid_f32(X, Y, 0.25)
    assert m == 100.0
    assert k.tolist() == [[2, 2, 4, 0]]   # sqrt(25/100) = 0.5, 0.5, 1, 0


@pytest.mark.parametrize("eps", [0.1, 0.03, 0.007])
def test_euclid_integer_grid_is_exact(eps):
    rng = np.random.default_rng(int(eps * 1000))
    X = rng.integers(0, 40, (30, 2)).astype(np.float32)
    Y = rng.integers(0, 40, (37, 2)).astype(np.float32)
    k, m = oracle.round_points_euclid_f32(X, Y, eps)
    d2 = ((X[:, None, :].astype(np.int64) - Y[None, :, :].astype(np.int64)) ** 2).sum(-1)
    assert m == float(d2.max())
    boundary = 0
    for b in range(30):
        for a in range(37):
            want, near = _exact_floor_sqrt_ratio(int(d2[b, a]), int(d2.max()), eps)
            if near:
                boundary += 1
                assert abs(int(k[b, a]) - want) <= 1
            else:
                assert k[b, a] == want, (b, a, d2[b, a])
    assert boundary < 60


def test_euclid_within_rounding_of_binary64_reference():
    X, Y = synth.uniform_points(200, 3, seed=9, n_a=150)
    eps = 0.01
    k, m = oracle.round_points_euclid_f32(X, Y, eps)
    d2 = ((X[:, None, :].astype(np.float64) - Y[None, :, :].astype(np.float64)) ** 2).sum(-1)
    x = np.sqrt(d2 / d2.max()) / eps
    ref = np.floor(x)
    diff = k.astype(np.int64) - ref.astype(np.int64)
    assert np.abs(diff).max() <= 1
    # a difference needs the exact value within binary32 rounding of an integer
    near = np.abs(x - np.rint(x)) < 1e-4
    assert (diff[~near] == 0).all()


def test_euclid_is_the_square_root_of_the_squared_cost():
    """Both variants are non-decreasing functions of the same binary32 d2:
    they share the maximum, and a pair with a smaller squared k never has a
    larger Euclidean k than a pair with a larger squared k."""
    X, Y = synth.uniform_points(80, 2, seed=3)
    ke, me = oracle.round_points_euclid_f32(X, Y, 0.01)
    ks, ms = oracle.round_points_f32(X, Y, 0.01)
    assert me == ms
    s, e = ks.ravel().astype(np.int64), ke.ravel().astype(np.int64)
    vals = np.unique(s)
    for lo, hi in zip(vals[:-1], vals[1:]):
        assert e[s == lo].max() <= e[s == hi].min()
    # and sqrt(c) >= c on [0, 1]: the Euclidean k is never the smaller
    assert (e >= s).all()


def test_l1_hand_values():
    X = np.array([[1, 1, 2, 0]], np.float32)                 # (1/4, 1/4, 1/2, 0)
    Y = np.array([[0, 2, 0, 2], [1, 1, 2, 0], [0, 0, 0, 4], [2, 2, 4, 0]], np.float32)
    k = oracle.round_l1_normalized_f32(X, Y, 0.25)
    # L1 = 1.5, 0, 2, 0 -> halves 0.75, 0, 1, 0 -> k = 3, 0, 4, 0
    assert k.tolist() == [[3, 0, 4, 0]]


@pytest.mark.parametrize("eps", [0.1, 0.05, 0.013])
def test_l1_dyadic_images_are_exact(eps):
    """Pixel values summing to 64: the normalised values are multiples of
    1/64 and every binary32 step is exact, so k = floor(L1 / 2 / eps) with
    exact rationals (away from binary64 ties at integers)."""
    rng = np.random.default_rng(int(eps * 1e4))
    n, d = 25, 16

    def imgs(count):
        out = np.zeros((count, d), np.float32)
        for i in range(count):
            cuts = np.sort(rng.integers(0, 65, d - 1))
            out[i] = np.diff(np.concatenate([[0], cuts, [64]]))
        return out

    X, Y = imgs(n), imgs(n + 3)
    k = oracle.round_l1_normalized_f32(X, Y, eps)
    e = Fraction(eps)
    for b in range(n):
        for a in range(n + 3):
            l1 = Fraction(int(np.abs(X[b] - Y[a]).sum()), 64)
            c = min(l1 / 2, Fraction(1))
            x = c / e
            want = math.floor(x)
            if abs(float(x) - round(float(x))) < 1e-9:
                assert abs(int(k[b, a]) - want) <= 1
            else:
                assert k[b, a] == want


def test_l1_within_rounding_of_binary64_reference():
    X = synth.digit_images(60, seed=2)
    Y = synth.digit_images(70, seed=3)
    eps = 0.01
    k = oracle.round_l1_normalized_f32(X, Y, eps)
    Xh = X.astype(np.float64) / X.astype(np.float64).sum(1, keepdims=True)
    Yh = Y.astype(np.float64) / Y.astype(np.float64).sum(1, keepdims=True)
    c = np.minimum(np.abs(Xh[:, None, :] - Yh[None, :, :]).sum(-1) / 2, 1.0)
    x = c / eps
    diff = k.astype(np.int64) - np.floor(x).astype(np.int64)
    assert np.abs(diff).max() <= 1
    near = np.abs(x - np.rint(x)) < 1e-3
    assert (diff[~near] == 0).all()


def test_l1_invariant_to_scaling_by_powers_of_two():
    X = synth.digit_images(20, seed=4)
    Y = synth.digit_images(25, seed=5)
    k1 = oracle.round_l1_normalized_f32(X, Y, 0.02)
    k2 = oracle.round_l1_normalized_f32(X * 4.0, Y * 0.5, 0.02)
    assert np.array_equal(k1, k2)
    # identical images cost 0; disjoint supports cost the maximum
    assert (np.diag(oracle.round_l1_normalized_f32(X, X, 0.02)) == 0).all()
    A = np.zeros((1, 4), np.float32)
    A[0, 0] = 1
    B = np.zeros((1, 4), np.float32)
    B[0, 3] = 5
    assert oracle.round_l1_normalized_f32(A, B, 0.02)[0, 0] == math.floor(1 / 0.02)


def test_l1_rejects_bad_images():
    good = np.ones((1, 4), np.float32)
    for bad in ([[1, -1, 1, 1]], [[0, 0, 0, 0]], [[1, float("nan"), 1, 1]],
                [[1, float("inf"), 1, 1]]):
        with pytest.raises(oracle.OracleError, match="range"):
            oracle.round_l1_normalized_f32(np.array(bad, np.float32), good, 0.1)
        with pytest.raises(oracle.OracleError, match="range"):
            oracle.round_l1_normalized_f32(good, np.array(bad, np.float32), 0.1)
