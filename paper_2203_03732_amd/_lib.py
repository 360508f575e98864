"""ctypes binding of libprot (include/prot.h). Argument marshalling only:
every step of the solver runs in the library's HIP kernels. PyTorch supplies
device memory and the current stream."""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libprot.so")

PROT_OK, PROT_PARTIAL = 0, 1
STATUS_NAMES = {0: "ok", 1: "partial", -1: "arg", -2: "range", -3: "eps", -4: "phase_bound",
                -5: "state", -6: "hip", -7: "nomem", -8: "unsupported"}
EPS_MODES = {"algorithmic": 0, "strict": 1}
ORIGINS = {"diag": 0, "zero": 1}


class ProtError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"prot error {code} ({STATUS_NAMES.get(code, '?')}): {msg}")
        self.code = code
        self.name = STATUS_NAMES.get(code, "?")


class Opts(ctypes.Structure):
    _fields_ = [("eps_mode", ctypes.c_int32), ("origin_mode", ctypes.c_int32),
                ("no_completion", ctypes.c_int32), ("cost_storage", ctypes.c_int32),
                ("k_type", ctypes.c_int32), ("check_warm", ctypes.c_int32),
                ("phase_bound", ctypes.c_int64), ("max_phases", ctypes.c_int64)]


COST_STORAGE = {"auto": 0, "matrix": 1, "on_the_fly": 2}
K_TYPES = {"auto": 0, "int16": 1, "uint8": 2}


class Stats(ctypes.Structure):
    _fields_ = [("phases", ctypes.c_int64), ("sum_free", ctypes.c_int64),
                ("rounds", ctypes.c_int64), ("max_rounds", ctypes.c_int64),
                ("scanned", ctypes.c_int64), ("matched_in_phases", ctypes.c_int64),
                ("completed_pairs", ctypes.c_int64), ("sum_k", ctypes.c_int64),
                ("threshold", ctypes.c_int64), ("kmax", ctypes.c_int32),
                ("status", ctypes.c_int32), ("cost", ctypes.c_double),
                ("cost_scale", ctypes.c_double), ("eps_internal", ctypes.c_double),
                ("ms_build", ctypes.c_double), ("ms_loop_kernel", ctypes.c_double),
                ("ms_total", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class OTStats(ctypes.Structure):
    _fields_ = [("theta", ctypes.c_double), ("copies_b", ctypes.c_int64),
                ("copies_a", ctypes.c_int64), ("repaired_mass", ctypes.c_double),
                ("loop", Stats)]

    def as_dict(self) -> dict:
        d = {name: getattr(self, name) for name, _ in self._fields_[:4]}
        d.update(self.loop.as_dict())
        return d


class BatchConfig(ctypes.Structure):
    """prot_batch_config: engine (0 auto, 1 LDS, 2 teams), team, cost_path
    (-1: the context's)."""
    _fields_ = [("engine", ctypes.c_int32), ("team", ctypes.c_int32),
                ("cost_path", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    ENGINES = {"auto": 0, "lds": 1, "teams": 2}

    @classmethod
    def from_dict(cls, d: dict) -> "BatchConfig":
        return cls(cls.ENGINES[d.get("engine", "auto")], int(d.get("team", 0)),
                   int(d.get("cost_path", -1)), 0)

    def as_dict(self) -> dict:
        names = {v: k for k, v in self.ENGINES.items()}
        return {"engine": names[self.engine], "team": self.team, "cost_path": self.cost_path}


class InstanceStats(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int64) for name in (
        "phases", "sum_free", "rounds", "max_rounds", "scanned", "matched_in_phases",
        "completed_pairs", "sum_k", "threshold")] + [
        ("status", ctypes.c_int32), ("kmax", ctypes.c_int32), ("cost", ctypes.c_double),
        ("cost_scale", ctypes.c_double)]


def instance_stats_from_bytes(buf) -> list[dict]:
    """Decode a byte buffer of prot_instance_stats records."""
    size = ctypes.sizeof(InstanceStats)
    raw = bytes(buf)
    out = []
    for i in range(len(raw) // size):
        rec = InstanceStats.from_buffer_copy(raw[i * size:(i + 1) * size])
        out.append({name: getattr(rec, name) for name, _ in InstanceStats._fields_})
    return out


_lib = None

EXPORTS = [
    "prot_ctx_create", "prot_ctx_destroy", "prot_set_stream", "prot_set_cost_path",
    "prot_reserve", "prot_pitch",
    "prot_threshold", "prot_max_n", "prot_round_costs", "prot_build_costs",
    "prot_solve_rounded", "prot_solve_cost", "prot_solve_points",
    "prot_round_costs_rect", "prot_build_costs_rect", "prot_solve_rounded_rect",
    "prot_solve_cost_rect", "prot_solve_points_rect", "prot_ot_solve", "prot_ot_solve_clustered",
    "prot_set_cost_metric",
    "prot_get_trace",
    "prot_get_round_times", "prot_loop_times", "prot_batch_max_n", "prot_batch_create", "prot_batch_destroy",
    "prot_batch_create_config", "prot_batch_autotune",
    "prot_batch_run", "prot_batch_capture", "prot_batch_replay", "prot_solve_batched_points",
    "prot_batch_loss_fwd", "prot_batch_loss_bwd", "prot_ctx_status", "prot_batch_status",
    "prot_ot_loss_fwd", "prot_ot_loss_bwd", "prot_ot_loss_fwd_static",
    "prot_status_string", "prot_last_error",
]


def load():
    """Load libprot.so (built in-tree by paper_2203_03732_amd.build). There
    is no fallback: without the library nothing in this package can run."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2203_03732_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    p, i32, i64, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "prot_ctx_create": (ctypes.c_int, [ctypes.POINTER(p), ctypes.c_int, p]),
        "prot_ctx_destroy": (ctypes.c_int, [p]),
        "prot_set_stream": (ctypes.c_int, [p, p]),
        "prot_set_cost_path": (ctypes.c_int, [p, i32]),
        "prot_reserve": (ctypes.c_int, [p, i64, i32]),
        "prot_pitch": (i64, [i64]),
        "prot_threshold": (i64, [f64, i64]),
        "prot_max_n": (i64, [p]),
        "prot_round_costs": (ctypes.c_int, [p, p, i64, i64, f64, p, i64]),
        "prot_build_costs": (ctypes.c_int, [p, p, p, i64, i32, f64, p, i64, p]),
        "prot_solve_rounded": (ctypes.c_int, [p, p, i64, i64, i64, ctypes.POINTER(Opts), i32,
                                              p, p, p, p, ctypes.POINTER(Stats)]),
        "prot_solve_cost": (ctypes.c_int, [p, p, i64, i64, f64, ctypes.POINTER(Opts),
                                           p, p, p, p, ctypes.POINTER(Stats)]),
        "prot_solve_points": (ctypes.c_int, [p, p, p, i64, i32, f64, ctypes.POINTER(Opts),
                                             p, p, p, p, ctypes.POINTER(Stats)]),
        "prot_round_costs_rect": (ctypes.c_int, [p, p, i64, i64, i64, f64, p, i64]),
        "prot_build_costs_rect": (ctypes.c_int, [p, p, i64, p, i64, i32, f64, p, i64, p]),
        "prot_solve_rounded_rect": (ctypes.c_int, [p, p, i64, i64, i64, i64,
                                                   ctypes.POINTER(Opts), i32, p, p, p, p,
                                                   ctypes.POINTER(Stats)]),
        "prot_solve_cost_rect": (ctypes.c_int, [p, p, i64, i64, i64, f64, ctypes.POINTER(Opts),
                                                p, p, p, p, ctypes.POINTER(Stats)]),
        "prot_solve_points_rect": (ctypes.c_int, [p, p, i64, p, i64, i32, f64,
                                                  ctypes.POINTER(Opts), p, p, p, p,
                                                  ctypes.POINTER(Stats)]),
        "prot_ot_solve": (ctypes.c_int, [p, p, i64, i64, i64, p, p, f64, ctypes.POINTER(Opts),
                                         p, i64, p, p, p, p, ctypes.POINTER(OTStats)]),
        "prot_ot_solve_clustered": (ctypes.c_int, [p, p, i64, i64, i64, p, p, f64,
                                                   ctypes.POINTER(Opts), p, i64, p, p, p, p,
                                                   ctypes.POINTER(OTStats)]),
        "prot_set_cost_metric": (ctypes.c_int, [p, i32]),
        "prot_get_trace": (i64, [p, p, i64]),
        "prot_get_round_times": (i64, [p, p, i64]),
        "prot_batch_max_n": (i32, []),
        "prot_batch_create_config": (ctypes.c_int, [p, i32, p, i32, f64, ctypes.POINTER(Opts),
                                                     ctypes.POINTER(BatchConfig), ctypes.POINTER(p)]),
        "prot_batch_autotune": (ctypes.c_int, [p, i32, p, i32, f64, ctypes.POINTER(Opts), p, p,
                                               i32, ctypes.POINTER(BatchConfig),
                                               ctypes.POINTER(f64), ctypes.POINTER(i32)]),
        "prot_batch_create": (ctypes.c_int, [p, i32, p, i32, f64, ctypes.POINTER(Opts),
                                             ctypes.POINTER(p)]),
        "prot_batch_destroy": (ctypes.c_int, [p]),
        "prot_batch_run": (ctypes.c_int, [p, p, p, p, p, p, p, p]),
        "prot_batch_capture": (ctypes.c_int, [p, p, p, p, p, p, p, p]),
        "prot_batch_replay": (ctypes.c_int, [p]),
        "prot_batch_loss_fwd": (ctypes.c_int, [p, p, p, p, p]),
        "prot_batch_loss_bwd": (ctypes.c_int, [p, p, p, p, p, p, p, p]),
        "prot_solve_batched_points": (ctypes.c_int, [p, i32, p, i32, p, p, f64,
                                                     ctypes.POINTER(Opts), p, p, p, p, p]),
        "prot_ctx_status": (ctypes.c_int, [p]),
        "prot_loop_times": (i32, [p, p, i32]),
        "prot_batch_status": (ctypes.c_int, [p]),
        "prot_ot_loss_fwd": (ctypes.c_int, [p, i32, i64, i32, p, p, p, p]),
        "prot_ot_loss_bwd": (ctypes.c_int, [p, i32, i64, i32, p, p, p, p, p, p]),
        "prot_ot_loss_fwd_static": (ctypes.c_int, [i32, i64, i32, p, p, p, p, p]),
        "prot_status_string": (ctypes.c_char_p, [ctypes.c_int]),
        "prot_last_error": (ctypes.c_char_p, [p]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def pitch(n: int) -> int:
    return int(load().prot_pitch(int(n)))


def threshold(eps: float, n: int) -> int:
    return int(load().prot_threshold(float(eps), int(n)))


@dataclass
class Result:
    mate_a: object
    mate_b: object
    y_a: object
    y_b: object
    status: str
    stats: dict = field(default_factory=dict)


@dataclass
class OTResult:
    """plan: n_b x n_a float64; duals in the two-cluster form of Lemma 4.1:
    per point the smaller dual of its copies and how many copies hold it."""
    plan: object
    y_b_lo: object
    y_b_nlo: object
    y_a_lo: object
    y_a_nlo: object
    status: str
    stats: dict = field(default_factory=dict)


def _torch():
    import torch
    return torch


def _dev_ptr(t, dtype, name, ndim=None):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if ndim is not None and t.dim() != ndim:
        raise ValueError(f"{name} must have {ndim} dimensions")
    return ctypes.c_void_p(t.data_ptr())


class Context:
    """One library context bound to a device; enqueues on torch's current
    stream at each call."""

    def __init__(self, device: int | None = None):
        torch = _torch()
        lib = load()
        self.device = torch.cuda.current_device() if device is None else int(device)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            stream = torch.cuda.current_stream().cuda_stream
            rc = lib.prot_ctx_create(ctypes.byref(h), self.device, ctypes.c_void_p(stream))
        if rc != 0:
            raise ProtError(rc, "prot_ctx_create failed")
        self._h = h
        self._lib = lib
        self._stream = stream  # the stream the library enqueues on

    def close(self):
        for plan in self.__dict__.pop("_plans", {}).values():
            plan.close()
        if getattr(self, "_h", None):
            self._lib.prot_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- helpers
    def _bind_stream(self):
        s = _torch().cuda.current_stream(self.device).cuda_stream
        if s != self._stream:
            self._lib.prot_set_stream(self._h, ctypes.c_void_p(s))
            self._stream = s

    def _check(self, rc: int, allow_bound: bool = False) -> int:
        """Raise ProtError for an error code; PROT_E_PHASE_BOUND passes when
        allow_bound (the outputs then hold the valid state reached)."""
        if rc < 0 and not (allow_bound and rc == -4):
            msg = self._lib.prot_last_error(self._h).decode()
            raise ProtError(rc, msg)
        return rc

    @staticmethod
    def _opts(eps_mode="algorithmic", origin="diag", complete=True, max_phases=0,
              storage="auto", k_type="auto", phase_bound=0, check_warm=False) -> Opts:
        o = Opts()
        o.k_type = K_TYPES[k_type]
        o.phase_bound = int(phase_bound)
        o.check_warm = 1 if check_warm else 0
        o.eps_mode = EPS_MODES[eps_mode]
        o.origin_mode = ORIGINS[origin]
        o.no_completion = 0 if complete else 1
        o.cost_storage = COST_STORAGE[storage]
        o.max_phases = int(max_phases)
        return o

    def _outputs(self, n, n_a=None):
        """mate_a, mate_b, y_a, y_b for n rows and n_a (default n) columns:
        views of one allocation, each starting on a 256-byte boundary."""
        torch = _torch()
        n_a = n if n_a is None else n_a
        pa, pb = -(-n_a // 64) * 64, -(-n // 64) * 64
        buf = torch.empty(2 * (pa + pb), dtype=torch.int32, device=f"cuda:{self.device}")
        return (buf[:n_a], buf[pa:pa + n], buf[pa + pb:pa + pb + n_a],
                buf[2 * pa + pb:2 * pa + pb + n])

    # -- API
    def reserve(self, n_max: int, with_matrix: bool = True):
        self._check(self._lib.prot_reserve(self._h, int(n_max), 1 if with_matrix else 0))

    def max_n(self) -> int:
        return int(self._lib.prot_max_n(self._h))

    def alloc_k(self, n: int, n_a: int | None = None):
        torch = _torch()
        n_a = n if n_a is None else n_a
        return torch.empty((n, pitch(n_a)), dtype=torch.int16, device=f"cuda:{self.device}")

    def round_costs(self, C, eps: float, k=None):
        """C: n_b x n_a row-major float32 (n_b rows of supply)."""
        torch = _torch()
        if C.dim() != 2 or C.stride(1) != 1:
            raise ValueError("C must be a row-major n_b x n_a float32 matrix")
        n_b, n_a = C.shape
        if k is None:
            k = self.alloc_k(n_b, n_a)
        self._bind_stream()
        self._check(self._lib.prot_round_costs_rect(
            self._h, _dev_ptr(C, torch.float32, "C", 2), n_b, n_a, C.stride(0), float(eps),
            _dev_ptr(k, torch.int16, "k", 2), k.stride(0)))
        return k

    COST_PATHS = {"direct": 0, "matrix_cores": 1, "auto": 2}

    def set_cost_path(self, path: str) -> None:
        """'auto' (default: the matrix cores from d = 48), 'direct' or
        'matrix_cores' for later point-set builds; all give the same result
        (include/prot.h, prot_set_cost_path)."""
        self._check(self._lib.prot_set_cost_path(self._h, self.COST_PATHS[path]))

    COST_METRICS = {"sqeuclidean": 0, "euclidean": 1, "l1_normalized": 2}

    def set_cost_metric(self, metric: str) -> None:
        """'sqeuclidean' (default), 'euclidean' or 'l1_normalized' for later
        single-instance point-set builds and solves (include/prot.h,
        prot_set_cost_metric)."""
        self._check(self._lib.prot_set_cost_metric(self._h, self.COST_METRICS[metric]))

    def build_costs(self, X, Y, eps: float, k=None):
        """X: n_b x d rows, Y: n_a x d columns (contiguous float32)."""
        torch = _torch()
        n_b, d = X.shape
        n_a = Y.shape[0]
        if Y.shape != (n_a, d) or not X.is_contiguous() or not Y.is_contiguous():
            raise ValueError("X and Y must be contiguous n_b x d and n_a x d float32")
        if k is None:
            k = self.alloc_k(n_b, n_a)
        m = torch.empty(1, dtype=torch.float32, device=f"cuda:{self.device}")
        self._bind_stream()
        self._check(self._lib.prot_build_costs_rect(
            self._h, _dev_ptr(X, torch.float32, "X", 2), n_b, _dev_ptr(Y, torch.float32, "Y", 2),
            n_a, d, float(eps), _dev_ptr(k, torch.int16, "k", 2), k.stride(0),
            _dev_ptr(m, torch.float32, "m")))
        return k, m

    def loop_times(self, count: int):
        """Device times (ms) of the last `count` phase-loop launches on this
        context, oldest first (prot_loop_times; synchronises): the timing of
        solves enqueued with stats=False."""
        import numpy as np
        out = np.zeros(max(int(count), 0), np.float32)
        m = self._lib.prot_loop_times(self._h, out.ctypes.data_as(ctypes.c_void_p), len(out))
        if m < 0:
            self._check(m)
        return out[:m].astype(np.float64)

    def status(self) -> str:
        """How the work last enqueued by a solve on this context ended
        (prot_ctx_status; synchronises): 'ok', 'partial' or 'phase_bound';
        raises ProtError for a failure the device reported."""
        return STATUS_NAMES[self._check(self._lib.prot_ctx_status(self._h), allow_bound=True)]

    def solve_rounded(self, k, T: int, n: int | None = None, *, n_a: int | None = None,
                      state=None, origin="diag", complete=True, max_phases=0,
                      phase_bound=0, check_warm=False, stats=True) -> Result:
        """k: n rows x ldk (ldk >= n_a) int16; n_a columns, default n (the
        unbalanced case of Section 3.3 when n_a > n). phase_bound: the
        watchdog (0: the safe bound, > 0: that many phases, < 0: off); a
        stop there raises ProtError('phase_bound') unless stats=False.
        check_warm: also check (I2) on a warm start. stats=False enqueues
        only (then call status())."""
        torch = _torch()
        n = k.shape[0] if n is None else int(n)
        n_a = n if n_a is None else int(n_a)
        if k.dim() != 2 or k.stride(1) != 1 or k.shape[1] < n_a or k.shape[0] < n:
            raise ValueError("k must be a row-major n x ldk int16 matrix, ldk >= n_a")
        if state is None:
            mate_a, mate_b, y_a, y_b = self._outputs(n, n_a)
            warm = 0
        else:
            mate_a, mate_b, y_a, y_b = (state[x].clone() for x in ("mate_a", "mate_b", "y_a", "y_b"))
            warm = 1
        st = Stats()
        o = self._opts(origin=origin, complete=complete, max_phases=max_phases,
                       phase_bound=phase_bound, check_warm=check_warm)
        self._bind_stream()
        rc = self._check(self._lib.prot_solve_rounded_rect(
            self._h, _dev_ptr(k, torch.int16, "k", 2), n, n_a, k.stride(0), int(T), ctypes.byref(o),
            warm, _dev_ptr(mate_a, torch.int32, "mate_a"), _dev_ptr(mate_b, torch.int32, "mate_b"),
            _dev_ptr(y_a, torch.int32, "y_a"), _dev_ptr(y_b, torch.int32, "y_b"),
            ctypes.byref(st) if stats else None), allow_bound=True)
        return Result(mate_a, mate_b, y_a, y_b, STATUS_NAMES[rc], st.as_dict() if stats else {})

    def ot_loss(self, X, Y, mate_b):
        """prot_ot_loss_fwd: X, Y (batch, n, d) float32, mate_b (batch, n)
        int32 (local column of each row, -1 unmatched) -> (batch,) float32
        loss (1/n) sum_b ||x_b - y_mate(b)||^2."""
        torch = _torch()
        if X.dim() != 3 or Y.shape != X.shape or mate_b.shape != X.shape[:2] or \
                not X.is_contiguous() or not Y.is_contiguous() or not mate_b.is_contiguous():
            raise ValueError("X, Y must be contiguous (batch, n, d) and mate_b (batch, n)")
        batch, n, d = X.shape
        loss = torch.empty(batch, dtype=torch.float32, device=X.device)
        self._bind_stream()
        self._check(self._lib.prot_ot_loss_fwd(
            self._h, batch, n, d, _dev_ptr(X, torch.float32, "X", 3),
            _dev_ptr(Y, torch.float32, "Y", 3), _dev_ptr(mate_b, torch.int32, "mate_b", 2),
            _dev_ptr(loss, torch.float32, "loss", 1)))
        return loss

    def ot_loss_grad(self, X, Y, mate_b, grad_loss):
        """prot_ot_loss_bwd: (dX, dY) of sum_i grad_loss[i] * L_i for the
        fixed matching mate_b."""
        torch = _torch()
        if X.dim() != 3 or Y.shape != X.shape or mate_b.shape != X.shape[:2] or \
                not X.is_contiguous() or not Y.is_contiguous() or not mate_b.is_contiguous():
            raise ValueError("X, Y must be contiguous (batch, n, d) and mate_b (batch, n)")
        batch, n, d = X.shape
        g = grad_loss.to(torch.float32).contiguous()
        dX, dY = torch.empty_like(X), torch.empty_like(Y)
        self._bind_stream()
        self._check(self._lib.prot_ot_loss_bwd(
            self._h, batch, n, d, _dev_ptr(X, torch.float32, "X", 3),
            _dev_ptr(Y, torch.float32, "Y", 3), _dev_ptr(mate_b, torch.int32, "mate_b", 2),
            _dev_ptr(g, torch.float32, "grad_loss", 1), _dev_ptr(dX, torch.float32, "dX", 3),
            _dev_ptr(dY, torch.float32, "dY", 3)))
        return dX, dY

    def solve_cost(self, C, eps: float, *, eps_mode="algorithmic", origin="diag",
                   complete=True, max_phases=0, k_type="auto") -> Result:
        """C: n_b x n_a row-major float32 in [0, 1], n_b <= n_a. k_type: the
        stored matrix's element type, 'auto', 'int16' or 'uint8'."""
        torch = _torch()
        if C.dim() != 2 or C.stride(1) != 1:
            raise ValueError("C must be a row-major n_b x n_a float32 matrix")
        n, n_a = C.shape
        mate_a, mate_b, y_a, y_b = self._outputs(n, n_a)
        st = Stats()
        o = self._opts(eps_mode, origin, complete, max_phases, k_type=k_type)
        self._bind_stream()
        rc = self._check(self._lib.prot_solve_cost_rect(
            self._h, _dev_ptr(C, torch.float32, "C", 2), n, n_a, C.stride(0), float(eps),
            ctypes.byref(o), _dev_ptr(mate_a, torch.int32, "mate_a"),
            _dev_ptr(mate_b, torch.int32, "mate_b"), _dev_ptr(y_a, torch.int32, "y_a"),
            _dev_ptr(y_b, torch.int32, "y_b"), ctypes.byref(st)))
        return Result(mate_a, mate_b, y_a, y_b, STATUS_NAMES[rc], st.as_dict())

    def solve_points(self, X, Y, eps: float, *, eps_mode="algorithmic", origin="diag",
                     complete=True, max_phases=0, storage="auto", k_type="auto",
                     phase_bound=0, stats=True) -> Result:
        """storage: 'auto', 'matrix' (build and scan the n x n matrix) or
        'on_the_fly' (d = 2, 3: no matrix, each examined cost recomputed from
        the points); k_type: the stored matrix's element type ('auto' = 'int16',
        or 'uint8' for floor(1/eps) <= 253: half the memory). All give the same
        result. stats=False enqueues only (no statistics, no synchronisation;
        Context.status() reports how the solve ended)."""
        torch = _torch()
        n, d = X.shape
        n_a = Y.shape[0]
        if Y.shape != (n_a, d) or not X.is_contiguous() or not Y.is_contiguous():
            raise ValueError("X and Y must be contiguous n_b x d and n_a x d float32")
        mate_a, mate_b, y_a, y_b = self._outputs(n, n_a)
        st = Stats()
        o = self._opts(eps_mode, origin, complete, max_phases, storage, k_type, phase_bound)
        self._bind_stream()
        rc = self._check(self._lib.prot_solve_points_rect(
            self._h, _dev_ptr(X, torch.float32, "X", 2), n, _dev_ptr(Y, torch.float32, "Y", 2),
            n_a, d, float(eps), ctypes.byref(o), _dev_ptr(mate_a, torch.int32, "mate_a"),
            _dev_ptr(mate_b, torch.int32, "mate_b"), _dev_ptr(y_a, torch.int32, "y_a"),
            _dev_ptr(y_b, torch.int32, "y_b"), ctypes.byref(st) if stats else None),
            allow_bound=True)
        return Result(mate_a, mate_b, y_a, y_b, STATUS_NAMES[rc], st.as_dict() if stats else {})

    def ot_solve(self, C, nu, mu, eps: float, *, eps_mode="algorithmic", origin="diag",
                 max_phases=0, plan=None, clustered=False) -> OTResult:
        """Optimal transport (Section 4) from supplies nu (rows of C) to
        demands mu (columns): C n_b x n_a float32 in [0, 1], nu and mu float64
        probability vectors, all on the device. clustered: keep each point's
        copies as two dual clusters (Lemma 4.1; prot_ot_solve_clustered)."""
        torch = _torch()
        if C.dim() != 2 or C.stride(1) != 1:
            raise ValueError("C must be a row-major n_b x n_a float32 matrix")
        n_b, n_a = C.shape
        if nu.shape != (n_b,) or mu.shape != (n_a,):
            raise ValueError("nu must have n_b entries and mu n_a")
        nu, mu = nu.contiguous(), mu.contiguous()  # kept alive across the call
        dev = f"cuda:{self.device}"
        if plan is None:
            plan = torch.empty((n_b, n_a), dtype=torch.float64, device=dev)
        if plan.shape != (n_b, n_a) or plan.stride(1) != 1:
            raise ValueError("plan must be a row-major n_b x n_a float64 matrix")
        kw = dict(dtype=torch.int32, device=dev)
        yb, nb_, ya, na_ = (torch.empty(n_b, **kw), torch.empty(n_b, **kw),
                            torch.empty(n_a, **kw), torch.empty(n_a, **kw))
        st = OTStats()
        o = self._opts(eps_mode, origin, True, max_phases)
        self._bind_stream()
        fn = self._lib.prot_ot_solve_clustered if clustered else self._lib.prot_ot_solve
        rc = self._check(fn(
            self._h, _dev_ptr(C, torch.float32, "C", 2), n_b, n_a, C.stride(0),
            _dev_ptr(nu, torch.float64, "nu", 1), _dev_ptr(mu, torch.float64, "mu", 1),
            float(eps), ctypes.byref(o),
            _dev_ptr(plan, torch.float64, "plan", 2), plan.stride(0),
            _dev_ptr(yb, torch.int32, "y_b_lo"), _dev_ptr(nb_, torch.int32, "y_b_nlo"),
            _dev_ptr(ya, torch.int32, "y_a_lo"), _dev_ptr(na_, torch.int32, "y_a_nlo"),
            ctypes.byref(st)))
        return OTResult(plan, yb, nb_, ya, na_, STATUS_NAMES[rc], st.as_dict())

    def round_times(self, cap: int = 65536):
        """(rounds, 3) int64: barrier arrival of the last workgroup, barrier
        exit, phase index; 100 MHz ticks. Empty unless the context was made
        with PROT_DEBUG_ROUND_TIMES=1."""
        import numpy as np
        buf = np.zeros((cap, 3), np.int64)
        m = int(self._lib.prot_get_round_times(self._h, buf.ctypes.data_as(ctypes.c_void_p), cap))
        if m < 0:
            raise ProtError(m, "prot_get_round_times failed")
        buf = buf[:m]
        return buf[buf[:, 1] != 0].copy()

    def cached_batch(self, ns, d: int, eps: float, **kw) -> "Batch":
        """A plan reused across calls with the same shapes and options."""
        key = (tuple(int(x) for x in ns), int(d), float(eps),
               tuple(sorted((k, repr(v)) for k, v in kw.items())))
        cache = self.__dict__.setdefault("_plans", {})
        if key not in cache:
            cache[key] = Batch(self, ns, d, eps, **kw)
        return cache[key]

    def batch(self, ns, d: int, eps: float, *, eps_mode="algorithmic", origin="diag",
              complete=True, max_phases=0, config=None) -> "Batch":
        """config: None (automatic), a dict {'engine': 'lds'|'teams'|'auto',
        'team': w, 'cost_path': -1|0|1} or a BatchConfig."""
        return Batch(self, ns, d, eps, eps_mode=eps_mode, origin=origin, complete=complete,
                     max_phases=max_phases, config=config)

    def autotune_batch(self, ns, d: int, eps: float, X, Y, *, reps: int = 3,
                       eps_mode="algorithmic", origin="diag", max_phases=0):
        """Time every batch configuration on X, Y (prot_batch_autotune);
        returns (best config dict, its mean ms, number of configurations)."""
        import numpy as np
        torch = _torch()
        ns = np.ascontiguousarray(np.asarray(ns, dtype=np.int64))
        o = self._opts(eps_mode, origin, True, max_phases)
        best, ms, tried = BatchConfig(), ctypes.c_double(), ctypes.c_int32()
        self._bind_stream()
        self._check(self._lib.prot_batch_autotune(
            self._h, len(ns), ns.ctypes.data_as(ctypes.c_void_p), int(d), float(eps),
            ctypes.byref(o), _dev_ptr(X, torch.float32, "X", 2), _dev_ptr(Y, torch.float32, "Y", 2),
            int(reps), ctypes.byref(best), ctypes.byref(ms), ctypes.byref(tried)))
        return best.as_dict(), ms.value, tried.value

    def solve_batched_points(self, ns, X, Y, eps: float, *, eps_mode="algorithmic",
                             origin="diag", complete=True, max_phases=0):
        """Instances packed row-wise: instance i is rows [o_i, o_i + ns[i]) of X
        and Y. Returns (mate_a, mate_b, y_a, y_b, per-instance stats list)."""
        import numpy as np
        torch = _torch()
        ns_arr = np.ascontiguousarray(np.asarray(ns, dtype=np.int64))
        total = int(ns_arr.sum())
        if X.shape[0] != total or Y.shape != X.shape or not X.is_contiguous() or not Y.is_contiguous():
            raise ValueError("X and Y must be contiguous (sum(ns), d) float32")
        d = X.shape[1]
        mate_a, mate_b, y_a, y_b = self._outputs(total)
        st = (InstanceStats * len(ns_arr))()
        o = self._opts(eps_mode, origin, complete, max_phases)
        self._bind_stream()
        self._check(self._lib.prot_solve_batched_points(
            self._h, len(ns_arr), ns_arr.ctypes.data_as(ctypes.c_void_p), d,
            _dev_ptr(X, torch.float32, "X", 2), _dev_ptr(Y, torch.float32, "Y", 2), float(eps),
            ctypes.byref(o), _dev_ptr(mate_a, torch.int32, "mate_a"),
            _dev_ptr(mate_b, torch.int32, "mate_b"), _dev_ptr(y_a, torch.int32, "y_a"),
            _dev_ptr(y_b, torch.int32, "y_b"), ctypes.cast(st, ctypes.c_void_p)))
        stats = [{name: getattr(r, name) for name, _ in InstanceStats._fields_} for r in st]
        return mate_a, mate_b, y_a, y_b, stats

    def trace(self, cap: int = 65536):
        import numpy as np
        buf = np.zeros((cap, 4), np.int64)
        m = int(self._lib.prot_get_trace(self._h, buf.ctypes.data_as(ctypes.c_void_p), cap))
        if m < 0:
            raise ProtError(m, "prot_get_trace failed")
        return buf[:m].copy()


class Batch:
    """A planned batch of point-set instances (prot_batch_*): run it directly,
    or capture it once into a HIP graph and replay it."""

    def __init__(self, ctx: Context, ns, d: int, eps: float, **kw):
        import numpy as np
        self.ctx = ctx
        self.ns = np.ascontiguousarray(np.asarray(ns, dtype=np.int64))
        self.total = int(self.ns.sum())
        self.d = int(d)
        h = ctypes.c_void_p()
        o = Context._opts(kw.get("eps_mode", "algorithmic"), kw.get("origin", "diag"),
                          kw.get("complete", True), kw.get("max_phases", 0))
        cfg = kw.get("config")
        cfg = None if cfg is None else (cfg if isinstance(cfg, BatchConfig)
                                        else BatchConfig.from_dict(cfg))
        ctx._check(ctx._lib.prot_batch_create_config(
            ctx._h, len(self.ns), self.ns.ctypes.data_as(ctypes.c_void_p), self.d, float(eps),
            ctypes.byref(o), ctypes.byref(cfg) if cfg is not None else None, ctypes.byref(h)))
        self.config = None if cfg is None else cfg.as_dict()
        self._h = h
        torch = _torch()
        self.mate_a, self.mate_b, self.y_a, self.y_b = ctx._outputs(self.total)
        self.stats_dev = torch.zeros(len(self.ns) * ctypes.sizeof(InstanceStats),
                                     dtype=torch.uint8, device=f"cuda:{ctx.device}")

    def _ptrs(self, X, Y):
        torch = _torch()
        if X.shape != (self.total, self.d) or Y.shape != X.shape or not X.is_contiguous() \
                or not Y.is_contiguous():
            raise ValueError("X and Y must be contiguous (sum(ns), d) float32")
        return (_dev_ptr(X, torch.float32, "X", 2), _dev_ptr(Y, torch.float32, "Y", 2),
                _dev_ptr(self.mate_a, torch.int32, "mate_a"),
                _dev_ptr(self.mate_b, torch.int32, "mate_b"),
                _dev_ptr(self.y_a, torch.int32, "y_a"), _dev_ptr(self.y_b, torch.int32, "y_b"),
                ctypes.c_void_p(self.stats_dev.data_ptr()))

    def run(self, X, Y, check=True):
        """Enqueue the batch; with check (default) wait for it and raise
        ProtError if the device reported a failure (prot_batch_status)."""
        self.ctx._bind_stream()
        self.ctx._check(self.ctx._lib.prot_batch_run(self._h, *self._ptrs(X, Y)))
        if check:
            self.status()

    def status(self) -> str:
        """How the last run or replay ended ('ok'; raises ProtError for a
        failure or a stop by the phase-bound watchdog). Synchronises."""
        self.ctx._bind_stream()
        return STATUS_NAMES[self.ctx._check(self.ctx._lib.prot_batch_status(self._h))]

    def capture(self, X, Y):
        self.ctx._bind_stream()
        self.ctx._check(self.ctx._lib.prot_batch_capture(self._h, *self._ptrs(X, Y)))

    def replay(self):
        self.ctx._bind_stream()
        self.ctx._check(self.ctx._lib.prot_batch_replay(self._h))

    def stats(self) -> list[dict]:
        return instance_stats_from_bytes(self.stats_dev.cpu().numpy().tobytes())

    def loss(self, X, Y, mate_b=None):
        """Per-instance (1/n) sum ||x_b - y_mate(b)||^2 as a float32 tensor."""
        torch = _torch()
        mate_b = self.mate_b if mate_b is None else mate_b
        out = torch.empty(len(self.ns), dtype=torch.float32, device=X.device)
        self.ctx._bind_stream()
        self.ctx._check(self.ctx._lib.prot_batch_loss_fwd(
            self._h, _dev_ptr(X, torch.float32, "X"), _dev_ptr(Y, torch.float32, "Y"),
            _dev_ptr(mate_b, torch.int32, "mate_b"), _dev_ptr(out, torch.float32, "loss")))
        return out

    def loss_grad(self, X, Y, grad_loss, mate_a=None, mate_b=None):
        """(dX, dY) of sum_i grad_loss[i] * L_i for the fixed matching."""
        torch = _torch()
        mate_a = self.mate_a if mate_a is None else mate_a
        mate_b = self.mate_b if mate_b is None else mate_b
        grad_loss = grad_loss.to(torch.float32).contiguous()
        dX, dY = torch.empty_like(X), torch.empty_like(Y)
        self.ctx._bind_stream()
        self.ctx._check(self.ctx._lib.prot_batch_loss_bwd(
            self._h, _dev_ptr(X, torch.float32, "X"), _dev_ptr(Y, torch.float32, "Y"),
            _dev_ptr(mate_a, torch.int32, "mate_a"), _dev_ptr(mate_b, torch.int32, "mate_b"),
            _dev_ptr(grad_loss, torch.float32, "grad_loss"), _dev_ptr(dX, torch.float32, "dX"),
            _dev_ptr(dY, torch.float32, "dY")))
        return dX, dY

    def close(self):
        if getattr(self, "_h", None):
            self.ctx._lib.prot_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_default: dict[int, Context] = {}


def ot_loss_static(X, Y, mate_b, loss=None):
    """prot_ot_loss_fwd_static: the loss of Context.ot_loss without a context
    and without any device allocation by the library (its partial sums live
    in a fixed device array; calls that overlap on one GPU race). X, Y
    (batch, n, d) float32, mate_b (batch, n) int32, loss (batch,) float32
    (allocated here by torch when not given); the current torch stream and
    device."""
    torch = _torch()
    if X.dim() != 3 or Y.shape != X.shape or mate_b.shape != X.shape[:2] or \
            not X.is_contiguous() or not Y.is_contiguous() or not mate_b.is_contiguous():
        raise ValueError("X, Y must be contiguous (batch, n, d) and mate_b (batch, n)")
    batch, n, d = X.shape
    if loss is None:
        loss = torch.empty(batch, dtype=torch.float32, device=X.device)
    lib = load()
    with torch.cuda.device(X.device):
        s = torch.cuda.current_stream(X.device).cuda_stream
        rc = lib.prot_ot_loss_fwd_static(
            batch, n, d, _dev_ptr(X, torch.float32, "X", 3), _dev_ptr(Y, torch.float32, "Y", 3),
            _dev_ptr(mate_b, torch.int32, "mate_b", 2), _dev_ptr(loss, torch.float32, "loss", 1),
            ctypes.c_void_p(s))
    if rc < 0:
        raise ProtError(rc, lib.prot_last_error(None).decode())
    return loss


def context(device: int | None = None) -> Context:
    torch = _torch()
    dev = torch.cuda.current_device() if device is None else int(device)
    if dev not in _default:
        _default[dev] = Context(dev)
    return _default[dev]
