"""CPU oracle for the push-relabel additive epsilon-approximation of the
assignment problem (Lahn, Raghvendra, Zhang, arXiv:2203.03732).

TEST INFRASTRUCTURE. Only the tests, the smoke check and the CPU-baseline
leg of the benchmark import this package. It shares no code with the GPU
library: the C file next to this one is compiled by gcc into its own shared
object and reached through ctypes.

Conventions (Section 2.1): rows of every matrix are supply vertices B,
columns are demand vertices A; rounded costs k and dual weights are integer
numbers of epsilon steps.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

ORIGIN = {"diag": 0, "zero": 1}
STATUS = {0: "ok", 1: "partial", -1: "arg", -2: "range", -3: "eps", -7: "nomem",
          -8: "state"}


class OracleError(RuntimeError):
    pass


def build() -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math, no contraction)."""
    tmp = _LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True, cwd=_HERE)
    os.replace(tmp, _LIB)
    return _LIB


class _Stats(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int64) for name in (
        "phases", "sum_free", "rounds", "max_rounds", "scanned",
        "matched_in_phases", "completed_pairs", "sum_k")]


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    # tests of the pins themselves load a deliberately broken copy
    override = os.environ.get("ORACLE_LIB_OVERRIDE")
    if not override and not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(override or _LIB)
    p, i64, i32, f64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    lib.orc_round_cost.argtypes = [p, i64, i64, i64, f64, p, i64]
    lib.orc_round_points_f32.argtypes = [p, p, i64, i64, i32, f64, p, i64, p]
    lib.orc_points_cost_f64.argtypes = [p, p, i64, i64, i32, f64, p, p, p]
    lib.orc_solve_rounded.argtypes = [p, i64, i64, i64, i32, i64, i32, i32,
                                      p, p, p, p, p, p, i64]
    lib.orc_solve_rounded_rect.argtypes = [p, i64, i64, i64, i64, i32, i64, i32, i32,
                                           p, p, p, p, p, p, i64]
    lib.orc_points_max_f32.argtypes = [p, p, i64, i64, i32, p]
    lib.orc_ot_scale.argtypes = [p, i64, p, i64, f64, p, p, p, p, p]
    lib.orc_round_points_euclid_f32.argtypes = [p, p, i64, i64, i32, f64, p, i64, p]
    lib.orc_round_l1_normalized_f32.argtypes = [p, p, i64, i64, i32, f64, p, i64]
    lib.orc_ot_solve.argtypes = [p, i64, i64, i64, p, p, f64, i32, i64, i32, p, p, p, p, p,
                                 p, p, p, i64]
    lib.orc_points_pairs_f32.argtypes = [p, p, i32, f64, ctypes.c_float, p, p, i64, p]
    lib.orc_ot_clustered_rounded.argtypes = [p, i64, i64, i64, p, p, i64, i32, i64, i32, i32,
                                             p, p, p, p, p, p, p, p, p, i64]
    lib.orc_ot_solve_clustered.argtypes = [p, i64, i64, i64, p, p, f64, i32, i64, i32, p, p,
                                           p, p, p, p, p, p, p, i64]
    lib.orc_solve_points_f32.argtypes = [p, p, i64, i64, i32, f64, i64, i32, i64, i32,
                                         p, p, p, p, p, p, i64, p]
    for fn in (lib.orc_solve_points_f32, lib.orc_round_cost, lib.orc_round_points_f32,
               lib.orc_points_cost_f64, lib.orc_solve_rounded, lib.orc_solve_rounded_rect,
               lib.orc_points_max_f32, lib.orc_ot_scale, lib.orc_ot_solve,
               lib.orc_round_points_euclid_f32, lib.orc_round_l1_normalized_f32,
               lib.orc_points_pairs_f32, lib.orc_ot_clustered_rounded,
               lib.orc_ot_solve_clustered):
        fn.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _check(rc: int, what: str) -> int:
    if rc < 0:
        raise OracleError(f"{what}: {STATUS.get(rc, rc)}")
    return rc


def threshold(eps: float, n: int) -> int:
    """Integer form of the stop test |B'| <= eps*n (Section 2.2)."""
    return int(math.floor(eps * n + 1e-9))


def round_cost(C: np.ndarray, eps: float) -> np.ndarray:
    """eq. (1) on a float32 cost matrix scaled to [0, 1]."""
    C = np.ascontiguousarray(C, dtype=np.float32)
    nb, na = C.shape
    k = np.empty((nb, na), dtype=np.int16)
    _check(_load().orc_round_cost(_ptr(C), nb, na, na, float(eps), _ptr(k), na),
           "round_cost")
    return k


def round_points_f32(X: np.ndarray, Y: np.ndarray, eps: float):
    """Squared Euclidean cost in binary32 (fma accumulation in coordinate
    order), normalised by its maximum and rounded by eq. (1) in binary64.
    Returns (k, m)."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    Y = np.ascontiguousarray(Y, dtype=np.float32)
    nb, d = X.shape
    na, d2 = Y.shape
    assert d == d2
    k = np.empty((nb, na), dtype=np.int16)
    m = np.zeros(1, dtype=np.float32)
    _check(_load().orc_round_points_f32(_ptr(X), _ptr(Y), nb, na, d, float(eps),
                                        _ptr(k), na, _ptr(m)), "round_points_f32")
    return k, float(m[0])


def round_points_euclid_f32(X: np.ndarray, Y: np.ndarray, eps: float):
    """Plain Euclidean cost (Section 5's synthetic workload): the binary32
    squared distance and maximum of round_points_f32, cost sqrt(d2 / m) in
    binary64, eq. (1). Returns (k, m)."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    Y = np.ascontiguousarray(Y, dtype=np.float32)
    nb, d = X.shape
    na = Y.shape[0]
    k = np.empty((nb, na), dtype=np.int16)
    m = np.zeros(1, dtype=np.float32)
    _check(_load().orc_round_points_euclid_f32(_ptr(X), _ptr(Y), nb, na, d, float(eps),
                                               _ptr(k), na, _ptr(m)), "round_points_euclid_f32")
    return k, float(m[0])


def round_l1_normalized_f32(X: np.ndarray, Y: np.ndarray, eps: float) -> np.ndarray:
    """Section 5's image cost: vectors normalised to sum 1, half their L1
    distance (binary32, coordinate order), eq. (1)."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    Y = np.ascontiguousarray(Y, dtype=np.float32)
    nb, d = X.shape
    na = Y.shape[0]
    k = np.empty((nb, na), dtype=np.int16)
    _check(_load().orc_round_l1_normalized_f32(_ptr(X), _ptr(Y), nb, na, d, float(eps),
                                               _ptr(k), na), "round_l1_normalized_f32")
    return k


def points_max_f32(X: np.ndarray, Y: np.ndarray) -> float:
    """The binary32 maximum squared distance of round_points_f32, without the
    matrix (for large n)."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    Y = np.ascontiguousarray(Y, dtype=np.float32)
    m = np.zeros(1, dtype=np.float32)
    _check(_load().orc_points_max_f32(_ptr(X), _ptr(Y), X.shape[0], Y.shape[0], X.shape[1],
                                      _ptr(m)), "points_max_f32")
    return float(m[0])


def points_pairs_f32(X: np.ndarray, Y: np.ndarray, eps: float, m: float, b_idx, a_idx):
    """Eq. (1) of round_points_f32 for the pairs (b_idx[i], a_idx[i]) only,
    given the maximum m."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    Y = np.ascontiguousarray(Y, dtype=np.float32)
    b_idx = np.ascontiguousarray(b_idx, dtype=np.int64)
    a_idx = np.ascontiguousarray(a_idx, dtype=np.int64)
    out = np.empty(len(b_idx), dtype=np.int16)
    _check(_load().orc_points_pairs_f32(_ptr(X), _ptr(Y), X.shape[1], float(eps),
                                        ctypes.c_float(m), _ptr(b_idx), _ptr(a_idx),
                                        len(b_idx), _ptr(out)), "points_pairs_f32")
    return out


def points_cost_f64(X: np.ndarray, Y: np.ndarray, eps: float | None = None,
                    want_c: bool = True):
    """Binary64 reference: c64 = d2 / max d2 and k64 = floor(c64 / eps).
    Returns (c64 or None, k64 or None, m64)."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    Y = np.ascontiguousarray(Y, dtype=np.float32)
    nb, d = X.shape
    na = Y.shape[0]
    c = np.empty((nb, na), dtype=np.float64) if want_c else None
    k = np.empty((nb, na), dtype=np.int16) if eps is not None else None
    m = np.zeros(1, dtype=np.float64)
    _check(_load().orc_points_cost_f64(
        _ptr(X), _ptr(Y), nb, na, d, float(eps if eps is not None else 0.5),
        _ptr(c) if c is not None else None, _ptr(k) if k is not None else None,
        _ptr(m)), "points_cost_f64")
    return c, k, float(m[0])


def solve_rounded(k: np.ndarray, T: int, origin: str = "diag",
                  max_phases: int = 0, state: dict | None = None,
                  complete: bool = True, trace: bool = False,
                  trace_cap: int = 1 << 20) -> dict:
    """Run the phase loop of Section 2.2 on rounded costs k (rows B, columns
    A, |B| <= |A|: the unbalanced case of Section 3.3 when k is not square).

    state, if given, is a dict with int32 arrays mate_a, mate_b, y_a, y_b to
    resume from (copied, not modified). Returns a dict with the final arrays,
    the status ('ok' or 'partial'), the stats and, if asked, the per-phase
    trace as an (phases, 4) array of (|B'|, rounds, scanned, |M'|)."""
    k = np.ascontiguousarray(k, dtype=np.int16)
    n_b, n_a = k.shape
    assert n_b <= n_a, "the unbalanced case needs |B| <= |A| (transpose k)"
    if state is None:
        mate_a = np.full(n_a, -1, np.int32)
        mate_b = np.full(n_b, -1, np.int32)
        y_a = np.zeros(n_a, np.int32)
        y_b = np.ones(n_b, np.int32)
        warm = 0
    else:
        mate_a = np.array(state["mate_a"], dtype=np.int32, copy=True)
        mate_b = np.array(state["mate_b"], dtype=np.int32, copy=True)
        y_a = np.array(state["y_a"], dtype=np.int32, copy=True)
        y_b = np.array(state["y_b"], dtype=np.int32, copy=True)
        warm = 1
    st = _Stats()
    tr = np.zeros((trace_cap, 4), np.int64) if trace else None
    rc = _check(_load().orc_solve_rounded_rect(
        _ptr(k), n_b, n_a, n_a, int(T), ORIGIN[origin], int(max_phases), warm,
        1 if complete else 0, _ptr(mate_a), _ptr(mate_b), _ptr(y_a), _ptr(y_b),
        ctypes.byref(st), _ptr(tr) if tr is not None else None,
        trace_cap if tr is not None else 0), "solve_rounded")
    stats = {name: int(getattr(st, name)) for name, _ in _Stats._fields_}
    out = dict(mate_a=mate_a, mate_b=mate_b, y_a=y_a, y_b=y_b,
               status=STATUS[rc], stats=stats)
    if tr is not None:
        out["trace"] = tr[:min(stats["phases"], trace_cap)].copy()
    return out


def solve_points(X: np.ndarray, Y: np.ndarray, eps: float, T: int | None = None,
                 origin: str = "diag", max_phases: int = 0, complete: bool = True,
                 trace: bool = False, trace_cap: int = 1 << 20) -> dict:
    """The phase loop on the rounded squared-Euclidean costs of point sets X
    (rows) and Y (columns) without storing the matrix: every rounded cost the
    loop examines is computed from the points with round_points_f32's
    arithmetic (the binary32 maximum m over all pairs first). T defaults to
    threshold(eps, n_b). Same results as solve_rounded on round_points_f32's
    matrix; the dict also holds m."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    Y = np.ascontiguousarray(Y, dtype=np.float32)
    n_b, d = X.shape
    n_a = Y.shape[0]
    assert Y.shape[1] == d and n_b <= n_a
    if T is None:
        T = threshold(eps, n_b)
    mate_a = np.full(n_a, -1, np.int32)
    mate_b = np.full(n_b, -1, np.int32)
    y_a = np.zeros(n_a, np.int32)
    y_b = np.ones(n_b, np.int32)
    m = np.zeros(1, dtype=np.float32)
    st = _Stats()
    tr = np.zeros((trace_cap, 4), np.int64) if trace else None
    rc = _check(_load().orc_solve_points_f32(
        _ptr(X), _ptr(Y), n_b, n_a, d, float(eps), int(T), ORIGIN[origin], int(max_phases),
        1 if complete else 0, _ptr(mate_a), _ptr(mate_b), _ptr(y_a), _ptr(y_b),
        ctypes.byref(st), _ptr(tr) if tr is not None else None,
        trace_cap if tr is not None else 0, _ptr(m)), "solve_points")
    stats = {name: int(getattr(st, name)) for name, _ in _Stats._fields_}
    out = dict(mate_a=mate_a, mate_b=mate_b, y_a=y_a, y_b=y_b, status=STATUS[rc],
               stats=stats, m=float(m[0]))
    if tr is not None:
        out["trace"] = tr[:min(stats["phases"], trace_cap)].copy()
    return out


def ot_scale(nu, mu, eps: float):
    """Section 4 scaling: (s, d, theta) with s_b = floor(theta nu_b) supply
    copies and d_a = ceil(theta mu_a) demand copies, theta = 4 max(n_b, n_a)/eps."""
    nu = np.ascontiguousarray(nu, dtype=np.float64)
    mu = np.ascontiguousarray(mu, dtype=np.float64)
    s = np.zeros(len(nu), np.int64)
    d = np.zeros(len(mu), np.int64)
    th = ctypes.c_double()
    cb, ca = ctypes.c_int64(), ctypes.c_int64()
    _check(_load().orc_ot_scale(_ptr(nu), len(nu), _ptr(mu), len(mu), float(eps), _ptr(s),
                                _ptr(d), ctypes.byref(th), ctypes.byref(cb), ctypes.byref(ca)),
           "ot_scale")
    return s, d, th.value


def ot_solve(C: np.ndarray, nu, mu, eps: float, origin: str = "diag", max_phases: int = 0,
             state: dict | None = None, trace: bool = False, trace_cap: int = 1 << 20) -> dict:
    """Section 4: approximate transport plan from supplies nu (rows of C) to
    demands mu (columns) through unit copies, with the free-copy dual raise.
    Returns the plan (n_b x n_a float64; None unless the loop finished), the
    copy-level mates and duals, the copy counts s and d, theta, the plan's
    cost, the mass moved by the feasibility repair, T, status and stats."""
    C = np.ascontiguousarray(C, dtype=np.float32)
    nu = np.ascontiguousarray(nu, dtype=np.float64)
    mu = np.ascontiguousarray(mu, dtype=np.float64)
    n_b, n_a = C.shape
    s, d, theta = ot_scale(nu, mu, eps)
    NB, NA = int(s.sum()), int(d.sum())
    if state is None:
        mate_a = np.full(NA, -1, np.int32)
        mate_b = np.full(NB, -1, np.int32)
        y_a = np.zeros(NA, np.int32)
        y_b = np.ones(NB, np.int32)
        warm = 0
    else:
        mate_a, mate_b, y_a, y_b = (np.array(state[x], dtype=np.int32, copy=True)
                                    for x in ("mate_a", "mate_b", "y_a", "y_b"))
        warm = 1
    plan = np.zeros((n_b, n_a), np.float64)
    info = np.zeros(4, np.float64)
    st = _Stats()
    tr = np.zeros((trace_cap, 4), np.int64) if trace else None
    rc = _check(_load().orc_ot_solve(
        _ptr(C), n_b, n_a, n_a, _ptr(nu), _ptr(mu), float(eps), ORIGIN[origin],
        int(max_phases), warm, _ptr(mate_a), _ptr(mate_b), _ptr(y_a), _ptr(y_b), _ptr(plan),
        ctypes.byref(st), _ptr(info), _ptr(tr) if tr is not None else None,
        trace_cap if tr is not None else 0), "ot_solve")
    stats = {name: int(getattr(st, name)) for name, _ in _Stats._fields_}
    out = dict(plan=plan if rc == 0 else None, mate_a=mate_a, mate_b=mate_b, y_a=y_a, y_b=y_b,
               s=s, d=d, theta=float(info[0]), cost=float(info[1]), repaired=float(info[2]),
               T=int(info[3]), status=STATUS[rc], stats=stats)
    if tr is not None:
        out["trace"] = tr[:min(stats["phases"], trace_cap)].copy()
    return out


# ---------------------------------------------------------------------------
# Section 4 with Lemma 4.1: the copies of every point kept as clusters (at
# most two dual levels per point). State in eps steps: Y[b] (top dual of b's
# copies, where its F[b] free copies sit), Z[a] (top dual of a's copies, G[a]
# of them free at 0), w[b, a, p] (pairs whose demand copy's level has parity
# p; Z[a] and Z[a] - 1 differ in parity).

_CLUSTER_KEYS = ("Y", "F", "Z", "G", "w")


def _cluster_state(n_b, n_a, state):
    if state is None:
        return (np.ones(n_b, np.int32), np.zeros(n_b, np.int64), np.zeros(n_a, np.int32),
                np.zeros(n_a, np.int64), np.zeros((n_b, n_a, 2), np.int64)), 0
    dt = (np.int32, np.int64, np.int32, np.int64, np.int64)
    return tuple(np.array(state[x], dtype=t, copy=True) for x, t in zip(_CLUSTER_KEYS, dt)), 1


def cluster_levels(k, Z):
    """The level of the demand copies in each parity slot: lev[a, p]."""
    Z = np.asarray(Z, np.int64)
    lev = np.empty((len(Z), 2), np.int64)
    for p in (0, 1):
        lev[:, p] = np.where((Z & 1) == p, Z, Z - 1)
    return lev


def cluster_counts(k, Y, Z, G, F, w):
    """Copies per dual level: (b_hi, b_lo, a_top, a_bottom) = copies of b at
    Y_b and at Y_b - 1, copies of a at Z_a and at Z_a - 1."""
    k = np.asarray(k, np.int64)
    lev = cluster_levels(k, Z)
    Y = np.asarray(Y, np.int64)
    b_hi = np.asarray(F, np.int64).copy()
    b_lo = np.zeros_like(b_hi)
    a_top = np.where(np.asarray(Z) == 0, np.asarray(G, np.int64), 0)
    a_bot = np.zeros_like(a_top)
    for p in (0, 1):
        yb = k - lev[None, :, p]
        hi = yb == Y[:, None]
        b_hi += (w[:, :, p] * hi).sum(1)
        b_lo += (w[:, :, p] * ~hi).sum(1)
        top = (lev[:, p] == np.asarray(Z, np.int64))
        a_top += (w[:, :, p].sum(0) * top)
        a_bot += (w[:, :, p].sum(0) * ~top)
    return b_hi, b_lo, a_top, a_bot


def ot_clustered_rounded(k: np.ndarray, s, d, T: int, origin: str = "diag",
                         max_phases: int = 0, complete: bool = True, state: dict | None = None,
                         want_last: bool = False, trace: bool = False,
                         trace_cap: int = 1 << 20) -> dict:
    """The clustered copies' phase loop on rounded costs k (n_b x n_a) with
    s[b] supply and d[a] demand copies per point. Returns the state (Y, F, Z,
    G, w), flow (pairs per point pair, completion included when complete),
    m_last (M' of the last phase, when want_last), status and stats."""
    k = np.ascontiguousarray(k, dtype=np.int16)
    n_b, n_a = k.shape
    s = np.ascontiguousarray(s, dtype=np.int64)
    d = np.ascontiguousarray(d, dtype=np.int64)
    (Y, F, Z, G, w), warm = _cluster_state(n_b, n_a, state)
    flow = np.zeros((n_b, n_a), np.int64)
    m_last = np.zeros((n_b, n_a), np.int64) if want_last else None
    st = _Stats()
    tr = np.zeros((trace_cap, 4), np.int64) if trace else None
    rc = _check(_load().orc_ot_clustered_rounded(
        _ptr(k), n_b, n_a, n_a, _ptr(s), _ptr(d), int(T), ORIGIN[origin], int(max_phases),
        warm, int(bool(complete)), _ptr(Y), _ptr(F), _ptr(Z), _ptr(G), _ptr(w), _ptr(flow),
        _ptr(m_last) if m_last is not None else None, ctypes.byref(st),
        _ptr(tr) if tr is not None else None, trace_cap if tr is not None else 0),
        "ot_clustered_rounded")
    stats = {name: int(getattr(st, name)) for name, _ in _Stats._fields_}
    out = dict(Y=Y, F=F, Z=Z, G=G, w=w, flow=flow, m_last=m_last, status=STATUS[rc],
               stats=stats)
    if tr is not None:
        out["trace"] = tr[:min(stats["phases"], trace_cap)].copy()
    return out


def ot_solve_clustered(C: np.ndarray, nu, mu, eps: float, origin: str = "diag",
                       max_phases: int = 0, state: dict | None = None, trace: bool = False,
                       trace_cap: int = 1 << 20) -> dict:
    """ot_solve with the copies kept as clusters: the plan (None unless the
    loop finished), the cluster state (Y, F, Z, G, w), the copies per dual
    level (b_hi, b_lo, a_top, a_bot), s, d, theta, cost, repaired, T, status
    and stats."""
    C = np.ascontiguousarray(C, dtype=np.float32)
    nu = np.ascontiguousarray(nu, dtype=np.float64)
    mu = np.ascontiguousarray(mu, dtype=np.float64)
    n_b, n_a = C.shape
    s, d, theta = ot_scale(nu, mu, eps)
    (Y, F, Z, G, w), warm = _cluster_state(n_b, n_a, state)
    plan = np.zeros((n_b, n_a), np.float64)
    info = np.zeros(4, np.float64)
    st = _Stats()
    tr = np.zeros((trace_cap, 4), np.int64) if trace else None
    rc = _check(_load().orc_ot_solve_clustered(
        _ptr(C), n_b, n_a, n_a, _ptr(nu), _ptr(mu), float(eps), ORIGIN[origin],
        int(max_phases), warm, _ptr(Y), _ptr(F), _ptr(Z), _ptr(G), _ptr(w), _ptr(plan),
        ctypes.byref(st), _ptr(info), _ptr(tr) if tr is not None else None,
        trace_cap if tr is not None else 0), "ot_solve_clustered")
    stats = {name: int(getattr(st, name)) for name, _ in _Stats._fields_}
    k = round_cost(C, eps)
    b_hi, b_lo, a_top, a_bot = cluster_counts(k, Y, Z, G, F, w)
    out = dict(plan=plan if rc == 0 else None, Y=Y, F=F, Z=Z, G=G, w=w, b_hi=b_hi, b_lo=b_lo,
               a_top=a_top, a_bot=a_bot, s=s, d=d, theta=float(info[0]),
               cost=float(info[1]), repaired=float(info[2]), T=int(info[3]),
               status=STATUS[rc], stats=stats)
    if tr is not None:
        out["trace"] = tr[:min(stats["phases"], trace_cap)].copy()
    return out


# ---------------------------------------------------------------------------
# Matching-based OT loss (not in the paper; the paper motivates using the
# transport plan and duals in learning, Section 1). For one instance with
# matching mate_b (row b -> column a):
#     L = (1/n) * sum_b ||x_b - y_{mate(b)}||^2
# The matching is piecewise constant in X and Y, so the gradient is that of
# the fixed plan P = (1/n) * permutation:
#     dL/dx_b = (2/n) (x_b - y_{mate(b)}),  dL/dy_a = (2/n) (y_a - x_{mate^-1(a)}).
# Rows left unmatched (no completion) contribute nothing.

def ot_loss(X: np.ndarray, Y: np.ndarray, mate_b: np.ndarray) -> float:
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    n = X.shape[0]
    total = 0.0
    for b in range(n):
        a = int(mate_b[b])
        if a >= 0:
            diff = X[b] - Y[a]
            total += float(diff @ diff)
    return total / n if n else 0.0


def ot_loss_grad(X: np.ndarray, Y: np.ndarray, mate_b: np.ndarray, g: float = 1.0):
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    n = X.shape[0]
    dX = np.zeros_like(X)
    dY = np.zeros_like(Y)
    for b in range(n):
        a = int(mate_b[b])
        if a >= 0:
            diff = X[b] - Y[a]
            dX[b] = 2.0 * g * diff / n
            dY[a] = -2.0 * g * diff / n
    return dX, dY
