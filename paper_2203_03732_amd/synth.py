"""Seeded synthetic inputs.

This module draws the random inputs that both the GPU library and its CPU
checker consume, so that both see identical arrays. It holds none of the
solver's arithmetic. All draws use numpy's PCG64 generator and float32.

Workloads (the shapes of the paper's experiments, Section 5):
  uniform_costs   n x n i.i.d. uniform costs in [0, 1)
  uniform_points  two sets of n points i.i.d. uniform in the unit cube
                  (the paper's synthetic workload draws 2-D points)
  gaussian_batch  independent instances of uneven n with standard normal
                  points, as in minibatch optimal transport
  shifted_gaussian_batch  equal-n instances, X ~ N(0, I), Y ~ N(shift, I)
  random_k        small random integer rounded-cost matrices for tests
  digit_images    28 x 28 nonnegative stroke images (784-vectors), a
                  stand-in with the shape and sparsity of handwritten-digit
                  scans (Section 5's image experiment; no dataset is used)
  transport_clouds  a transport instance: supply points uniform in the unit
                  square, demand points uniform in the square shifted by
                  (shift, 0), squared distances scaled to max 1, and random
                  masses (uniform in [0.05, 1.05), normalised)
"""
from __future__ import annotations

import numpy as np


def uniform_costs(n: int, seed: int = 0, n_a: int | None = None) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.random((n, n if n_a is None else n_a), dtype=np.float32)


def uniform_points(n: int, d: int = 2, seed: int = 0, n_a: int | None = None):
    rng = np.random.default_rng(seed)
    X = rng.random((n, d), dtype=np.float32)
    Y = rng.random((n if n_a is None else n_a, d), dtype=np.float32)
    return X, Y


def gaussian_batch(batch: int = 512, n_lo: int = 64, n_hi: int = 1024,
                   d: int = 16, seed: int = 0):
    """Returns (ns, [X_i], [Y_i]) with n_i uniform in [n_lo, n_hi]."""
    rng = np.random.default_rng(seed)
    ns = rng.integers(n_lo, n_hi + 1, batch)
    Xs, Ys = [], []
    for n in ns:
        Xs.append(rng.standard_normal((int(n), d), dtype=np.float32))
        Ys.append(rng.standard_normal((int(n), d), dtype=np.float32))
    return [int(n) for n in ns], Xs, Ys


def shifted_gaussian_batch(batch: int = 64, n: int = 2048, d: int = 64,
                           shift: float = 0.5, seed: int = 0):
    """Returns (X, Y) of shape (batch, n, d): X ~ N(0, I), Y ~ N(shift, I)."""
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((batch, n, d), dtype=np.float32)
    Y = rng.standard_normal((batch, n, d), dtype=np.float32) + np.float32(shift)
    return X, Y


def random_k(n: int, kmax: int, seed: int = 0, n_a: int | None = None) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.integers(0, kmax + 1, (n, n if n_a is None else n_a)).astype(np.int16)


def transport_clouds(n_b: int, n_a: int, seed: int = 0, shift: float = 1.0):
    """(C, nu, mu): C float32 n_b x n_a in [0, 1], nu and mu float64
    probability vectors. The costs are input data here (squared distances
    in binary64, scaled by their maximum, rounded to binary32)."""
    rng = np.random.default_rng(seed)
    X = rng.random((n_b, 2))
    Y = rng.random((n_a, 2)) + np.array([shift, 0.0])
    C = ((X[:, None, :] - Y[None, :, :]) ** 2).sum(-1)
    C = (C / C.max()).astype(np.float32)
    nu = rng.random(n_b) + 0.05
    mu = rng.random(n_a) + 0.05
    return C, nu / nu.sum(), mu / mu.sum()


def digit_images(n: int, seed: int = 0) -> np.ndarray:
    """n x 784 float32 images: 2 to 4 random strokes (line segments in the
    central 20 x 20 box, drawn with a 3 x 3 brush), intensities in (0.6, 1],
    about a fifth of the pixels nonzero."""
    rng = np.random.default_rng(seed)
    out = np.zeros((n, 28, 28), np.float32)
    t = np.linspace(0.0, 1.0, 40)
    for i in range(n):
        img = out[i]
        for _ in range(int(rng.integers(2, 5))):
            p0, p1 = rng.uniform(4, 24, 2), rng.uniform(4, 24, 2)
            rr = np.rint(p0[0] + (p1[0] - p0[0]) * t).astype(int)
            cc = np.rint(p0[1] + (p1[1] - p0[1]) * t).astype(int)
            for dr in (-1, 0, 1):
                for dc in (-1, 0, 1):
                    img[np.clip(rr + dr, 0, 27), np.clip(cc + dc, 0, 27)] = 1.0
        nz = img > 0
        img[nz] *= rng.uniform(0.6, 1.0, int(nz.sum())).astype(np.float32)
    return out.reshape(n, 784)
