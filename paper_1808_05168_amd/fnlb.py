"""Python binding of libfnlb (include/fnlb.h): argument marshalling only.

Device memory for the state, the accumulators and the workspace is allocated
with torch on the GPU and handed to the library as raw pointers; the library
enqueues its kernels on the current torch stream of that device.  Every step
of the method runs in the library's HIP kernels; there is no host fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Iterable, List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfnlb.so")

FNLB_OK = 0
FP64, FP32_DEV = 0, 1
ASTAR, WALL_UZ_FIX, NOISE_LOC, FORCE_LITERAL, NO_GRAPH, SAMPLE_VELOCITY = 1, 2, 4, 8, 16, 32
TWO_STEP, ONE_STEP = 64, 128
DEFAULT_FLAGS = ASTAR | WALL_UZ_FIX
FIELD_C, FIELD_RHO, FIELD_UX, FIELD_UZ = 0, 1, 2, 3


class ReplicaParams(ctypes.Structure):
    _fields_ = [("Lx", ctypes.c_int32), ("Lz", ctypes.c_int32),
                ("rho0", ctypes.c_double), ("grad_c0", ctypes.c_double),
                ("kT", ctypes.c_double), ("G", ctypes.c_double),
                ("tau_d", ctypes.c_double), ("tau_s", ctypes.c_double),
                ("tau_e", ctypes.c_double), ("tau_q", ctypes.c_double),
                ("tau_eps", ctypes.c_double), ("seed", ctypes.c_uint64)]


class Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("sample_every", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("chunk_rows", ctypes.c_int32)]


class FnlbError(RuntimeError):
    pass


_lib = None
EXPORTS = ["fnlb_bytes_required", "fnlb_init", "fnlb_step", "fnlb_autotune",
           "fnlb_accumulate_structure_factor", "fnlb_read_structure_factor",
           "fnlb_read_pressure", "fnlb_read_populations", "fnlb_write_populations",
           "fnlb_reset_accumulators", "fnlb_get_time", "fnlb_set_time", "fnlb_destroy",
           "fnlb_strerror", "fnlb_adjoint_bytes_required", "fnlb_sq_misfit_gradient",
           "fnlb_checkpoint_bytes", "fnlb_save", "fnlb_load", "fnlb_pressure_misfit_gradient",
           "fnlb_build_id", "fnlb_init_static_work", "fnlb_reinit", "fnlb_sq_misfit",
           "fnlb_pressure_misfit", "fnlb_misfit_backward", "fnlb_step_vjp",
           "fnlb_launch_config", "fnlb_tune_lookup", "fnlb_tune_cache_save",
           "fnlb_tune_cache_load"]
STATIC_WORK_BYTES = 128 << 20  # FNLB_STATIC_WORK_BYTES


def load(path: str = LIB_PATH):
    """Loads libfnlb.so; raises if it has not been built, or if it was built
    from other sources than the ones next to it (a stale build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FnlbError(f"{path} not found: build it with `python -m paper_1808_05168_amd.build`")
    # torch brings its own HIP runtime; it must be the one in the process
    # before the library's first HIP call, or torch later finds no GPU
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    lib.fnlb_build_id.restype = ctypes.c_char_p
    from . import build as _build
    built, current = lib.fnlb_build_id().decode(), _build.source_id()
    if built != current:
        raise FnlbError(f"{path} was built from other sources (build id {built}, sources "
                        f"{current}): rebuild it with `python -m paper_1808_05168_amd.build`")
    vp, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)
    i64p = ctypes.POINTER(ctypes.c_int64)
    szp = ctypes.POINTER(ctypes.c_size_t)
    rp, op = ctypes.POINTER(ReplicaParams), ctypes.POINTER(Options)
    lib.fnlb_bytes_required.argtypes = [rp, ctypes.c_int32, op, szp, szp, szp]
    lib.fnlb_init.argtypes = [rp, ctypes.c_int32, op, vp, ctypes.c_size_t, vp, ctypes.c_size_t,
                              vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    lib.fnlb_init_static_work.argtypes = [rp, ctypes.c_int32, op, vp, ctypes.c_size_t, vp,
                                          ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    lib.fnlb_step.argtypes = [vp, ctypes.c_int64]
    lib.fnlb_autotune.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
    lib.fnlb_launch_config.argtypes = [vp, ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(ctypes.c_int32)]
    i32p = ctypes.POINTER(ctypes.c_int32)
    lib.fnlb_tune_lookup.argtypes = [rp, ctypes.c_int32, ctypes.c_int32, i32p, i32p, i32p]
    lib.fnlb_tune_cache_save.argtypes = [ctypes.c_char_p]
    lib.fnlb_tune_cache_load.argtypes = [ctypes.c_char_p]
    lib.fnlb_accumulate_structure_factor.argtypes = [vp]
    lib.fnlb_read_structure_factor.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, dp, dp, dp,
                                               i64p]
    lib.fnlb_read_pressure.argtypes = [vp, ctypes.c_int32, dp, dp, dp, i64p]
    lib.fnlb_read_populations.argtypes = [vp, ctypes.c_int32, dp]
    lib.fnlb_write_populations.argtypes = [vp, ctypes.c_int32, dp]
    lib.fnlb_reset_accumulators.argtypes = [vp]
    lib.fnlb_get_time.argtypes = [vp, i64p]
    lib.fnlb_set_time.argtypes = [vp, ctypes.c_int64]
    lib.fnlb_destroy.argtypes = [vp]
    lib.fnlb_adjoint_bytes_required.argtypes = [vp, ctypes.c_int64, ctypes.c_int32, szp]
    lib.fnlb_sq_misfit_gradient.argtypes = [vp, ctypes.c_int32, dp, dp, ctypes.c_int64,
                                            ctypes.c_int32, vp, ctypes.c_size_t, dp, dp]
    lib.fnlb_pressure_misfit_gradient.argtypes = [vp, dp, dp, ctypes.c_int64, ctypes.c_int32,
                                                  vp, ctypes.c_size_t, dp, dp]
    lib.fnlb_sq_misfit.argtypes = [vp, ctypes.c_int32, dp, dp, ctypes.c_int64, ctypes.c_int32,
                                   vp, ctypes.c_size_t, dp]
    lib.fnlb_pressure_misfit.argtypes = [vp, dp, dp, ctypes.c_int64, ctypes.c_int32, vp,
                                         ctypes.c_size_t, dp]
    lib.fnlb_misfit_backward.argtypes = [vp, vp, ctypes.c_size_t, dp]
    lib.fnlb_step_vjp.argtypes = [vp, dp, dp, dp, vp, ctypes.c_size_t]
    lib.fnlb_reinit.argtypes = [vp, rp, ctypes.c_int32]
    lib.fnlb_checkpoint_bytes.argtypes = [vp, szp]
    lib.fnlb_save.argtypes = [vp, vp, ctypes.c_size_t]
    lib.fnlb_load.argtypes = [vp, vp, ctypes.c_size_t]
    lib.fnlb_strerror.argtypes = [ctypes.c_int]
    lib.fnlb_strerror.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(rc: int, what: str) -> None:
    if rc != FNLB_OK:
        msg = load().fnlb_strerror(rc).decode()
        raise FnlbError(f"{what} failed: {msg} ({rc})")


def _dp(a: Optional[np.ndarray]):
    if a is None:
        return None
    if a.dtype != np.float64 or not a.flags.c_contiguous:
        raise TypeError("expected a C-contiguous float64 array")
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def replica_params(reps: Sequence) -> ctypes.Array:
    arr = (ReplicaParams * len(reps))()
    for i, r in enumerate(reps):
        arr[i] = ReplicaParams(r.Lx, r.Lz, r.rho0, r.grad_c0, r.kT, r.G, r.tau_d, r.tau_s,
                               r.tau_e, r.tau_q, r.tau_eps, r.seed & ((1 << 64) - 1))
    return arr


def bytes_required(reps: Sequence, precision: int = FP64, sample_every: int = 0,
                   flags: int = DEFAULT_FLAGS, chunk_rows: int = 0):
    lib = load()
    p = replica_params(reps)
    o = Options(precision, sample_every, flags, chunk_rows)
    s, a, w = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
    _check(lib.fnlb_bytes_required(p, len(reps), ctypes.byref(o), ctypes.byref(s),
                                   ctypes.byref(a), ctypes.byref(w)), "fnlb_bytes_required")
    return s.value, a.value, w.value


def tune_lookup(reps: Sequence, precision: int):
    """The autotuner's stored (steps per launch, rows per work item) for these
    replicas and precision, or None."""
    f, k, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(load().fnlb_tune_lookup(replica_params(reps), len(reps), precision, ctypes.byref(f),
                                   ctypes.byref(k), ctypes.byref(c)), "fnlb_tune_lookup")
    return (int(k.value), int(c.value)) if f.value else None


def tune_cache_save(path: str) -> None:
    """Writes the autotuner's choices of this process to a text file."""
    _check(load().fnlb_tune_cache_save(os.fsencode(path)), "fnlb_tune_cache_save")


def tune_cache_load(path: str) -> None:
    """Adds a tuning file's choices for the current GPU architecture."""
    _check(load().fnlb_tune_cache_load(os.fsencode(path)), "fnlb_tune_cache_load")


class Lattice:
    """A batch of one or more replicas on one GPU.

    reps: objects with the fields of ``fnlb_replica_params`` (e.g.
    ``workloads.Replica``).  precision: FP64 or FP32_DEV.  static_work: create
    the handle with ``fnlb_init_static_work`` (the library's static workspace
    instead of a torch-allocated one; steps launch without graphs; one such
    handle per GPU at a time).
    """

    def __init__(self, reps: Iterable, precision: int = FP64, sample_every: int = 0,
                 flags: int = DEFAULT_FLAGS, chunk_rows: int = 0, device: str = "cuda:0",
                 static_work: bool = False):
        import torch
        self.reps: List = list(reps)
        self.precision = precision
        self.sample_every = sample_every
        self.flags = flags
        lib = load()
        self._lib = lib
        self._params = replica_params(self.reps)
        self._opts = Options(precision, sample_every, flags, chunk_rows)
        sb, ab, wb = bytes_required(self.reps, precision, sample_every, flags, chunk_rows)
        self.device = torch.device(device)
        # torch's caching allocator returns 512-byte aligned blocks
        self.state = torch.empty(sb, dtype=torch.uint8, device=self.device)
        self.accum = torch.empty(ab, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        if static_work:
            self.work = None
            with torch.cuda.device(self.device):
                _check(lib.fnlb_init_static_work(
                    self._params, len(self.reps), ctypes.byref(self._opts),
                    ctypes.c_void_p(self.state.data_ptr()), sb,
                    ctypes.c_void_p(self.accum.data_ptr()), ab,
                    ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)),
                    "fnlb_init_static_work")
        else:
            self.work = torch.empty(wb, dtype=torch.uint8, device=self.device)
            _check(lib.fnlb_init(self._params, len(self.reps), ctypes.byref(self._opts),
                                 ctypes.c_void_p(self.state.data_ptr()), sb,
                                 ctypes.c_void_p(self.accum.data_ptr()), ab,
                                 ctypes.c_void_p(self.work.data_ptr()), wb,
                                 ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)),
                   "fnlb_init")
        self._h = h
        self._adj_ws = None       # adjoint workspace, kept between forward and backward
        self._misfit_token = 0    # counts forward sweeps (and reinits) of this handle

    # -- lifetime --
    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            # finish the handle's work before its graphs go and torch may
            # hand its buffers to someone else
            self.stream.synchronize()
            self._lib.fnlb_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- the method --
    def step(self, n: int = 1) -> None:
        _check(self._lib.fnlb_step(self._h, int(n)), "fnlb_step")

    def launch_config(self):
        """(steps per launch, rows per work item) the handle uses."""
        k, c = ctypes.c_int32(), ctypes.c_int32()
        _check(self._lib.fnlb_launch_config(self._h, ctypes.byref(k), ctypes.byref(c)),
               "fnlb_launch_config")
        return int(k.value), int(c.value)

    def autotune(self, steps_per_trial: int = 20) -> int:
        """Picks the fastest step kernel and row-range length; returns the rows."""
        c = ctypes.c_int32()
        _check(self._lib.fnlb_autotune(self._h, int(steps_per_trial), ctypes.byref(c)),
               "fnlb_autotune")
        return int(c.value)

    def reinit(self, reps: Iterable) -> None:
        """New parameters and seeds for the same shapes; back to the rest state
        at t = 0 with cleared accumulators (buffers and graphs are kept)."""
        reps = list(reps)
        p = replica_params(reps)
        _check(self._lib.fnlb_reinit(self._h, p, len(reps)), "fnlb_reinit")
        self.reps, self._params = reps, p
        self._misfit_token += 1

    def _adj_workspace(self, horizon: int, ckpt_every: int):
        import torch
        nb = ctypes.c_size_t()
        _check(self._lib.fnlb_adjoint_bytes_required(self._h, int(horizon), int(ckpt_every),
                                                     ctypes.byref(nb)),
               "fnlb_adjoint_bytes_required")
        if self._adj_ws is None or self._adj_ws.numel() != nb.value:
            self._adj_ws = None
            self._adj_ws = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
        return ctypes.c_void_p(self._adj_ws.data_ptr()), nb.value

    def _targets(self, target, weight, pressure: bool):
        r = self.reps[0]
        shape = (r.Lz,) if pressure else (r.Lz, r.Lx // 2 + 1)
        return (np.ascontiguousarray(target, dtype=np.float64).reshape(shape),
                np.ascontiguousarray(weight, dtype=np.float64).reshape(shape))

    def sq_misfit(self, S_target: np.ndarray, weight: np.ndarray, horizon: int,
                  ckpt_every: int = 100, field: int = FIELD_C) -> float:
        """J = sum_q w_q (S(q) - S*(q))^2 over `horizon` steps from the current
        state (forward sweep only; misfit_backward() differentiates it)."""
        St, w = self._targets(S_target, weight, False)
        ws, nb = self._adj_workspace(horizon, ckpt_every)
        J = ctypes.c_double()
        _check(self._lib.fnlb_sq_misfit(self._h, field, _dp(St), _dp(w), int(horizon),
                                        int(ckpt_every), ws, nb, ctypes.byref(J)),
               "fnlb_sq_misfit")
        self._misfit_token += 1
        return J.value

    def pressure_misfit(self, P_target: np.ndarray, weight: np.ndarray, horizon: int,
                        ckpt_every: int = 100) -> float:
        """J = sum_j w_j (Pbar_j - P*_j)^2 over `horizon` steps from the current
        state (forward sweep only; misfit_backward() differentiates it)."""
        Pt, w = self._targets(P_target, weight, True)
        ws, nb = self._adj_workspace(horizon, ckpt_every)
        J = ctypes.c_double()
        _check(self._lib.fnlb_pressure_misfit(self._h, _dp(Pt), _dp(w), int(horizon),
                                              int(ckpt_every), ws, nb, ctypes.byref(J)),
               "fnlb_pressure_misfit")
        self._misfit_token += 1
        return J.value

    def misfit_backward(self) -> np.ndarray:
        """dJ/d(tau_s, tau_d, G) of the last sq_misfit / pressure_misfit."""
        if self._adj_ws is None:
            raise FnlbError("misfit_backward needs a preceding sq_misfit or pressure_misfit")
        g = np.zeros(3)
        _check(self._lib.fnlb_misfit_backward(self._h, ctypes.c_void_p(self._adj_ws.data_ptr()),
                                              self._adj_ws.numel(), _dp(g)),
               "fnlb_misfit_backward")
        return g

    def sq_misfit_gradient(self, S_target: np.ndarray, weight: np.ndarray, horizon: int,
                           ckpt_every: int = 100, field: int = FIELD_C):
        """(J, dJ/d(tau_s, tau_d, G)) of J = sum_q w_q (S(q) - S*(q))^2 over
        `horizon` steps from the current state, by the adjoint of the step."""
        St, w = self._targets(S_target, weight, False)
        ws, nb = self._adj_workspace(horizon, ckpt_every)
        J = ctypes.c_double()
        g = np.zeros(3)
        _check(self._lib.fnlb_sq_misfit_gradient(self._h, field, _dp(St), _dp(w), int(horizon),
                                                 int(ckpt_every), ws, nb, ctypes.byref(J),
                                                 _dp(g)),
               "fnlb_sq_misfit_gradient")
        self._misfit_token += 1
        return J.value, g

    def pressure_misfit_gradient(self, P_target: np.ndarray, weight: np.ndarray, horizon: int,
                                 ckpt_every: int = 100):
        """(J, dJ/d(tau_s, tau_d, G)) of J = sum_j w_j (Pbar_j - P*_j)^2 over
        `horizon` steps from the current state (Pbar_j: time-averaged row means
        of P - P_ref), by the adjoint of the step."""
        Pt, w = self._targets(P_target, weight, True)
        ws, nb = self._adj_workspace(horizon, ckpt_every)
        J = ctypes.c_double()
        g = np.zeros(3)
        _check(self._lib.fnlb_pressure_misfit_gradient(self._h, _dp(Pt), _dp(w), int(horizon),
                                                       int(ckpt_every), ws, nb,
                                                       ctypes.byref(J), _dp(g)),
               "fnlb_pressure_misfit_gradient")
        self._misfit_token += 1
        return J.value, g

    def step_vjp(self, mu_next: np.ndarray):
        """(mu, dtheta) of one step from the current state: mu = (df(t+1)/df(t))^T
        mu_next and dtheta = mu_next . df(t+1)/d(tau_s, tau_d, G), arrays in the
        layout of read_populations."""
        r = self.reps[0]
        y = np.ascontiguousarray(mu_next, dtype=np.float64)
        if y.shape != (2, 9, r.Lz, r.Lx):
            raise ValueError(f"cotangent of shape {y.shape}, expected {(2, 9, r.Lz, r.Lx)}")
        mu = np.empty_like(y)
        dth = np.zeros(3)
        ws, nb = self._adj_workspace(1, 1)
        _check(self._lib.fnlb_step_vjp(self._h, _dp(y), _dp(mu), _dp(dth), ws, nb),
               "fnlb_step_vjp")
        return mu, dth

    def accumulate_structure_factor(self) -> None:
        _check(self._lib.fnlb_accumulate_structure_factor(self._h),
               "fnlb_accumulate_structure_factor")

    def read_structure_factor(self, rep: int = 0, field: int = FIELD_C):
        r = self.reps[rep]
        shape = (r.Lz, r.Lx // 2 + 1)
        a2, re, im = np.empty(shape), np.empty(shape), np.empty(shape)
        n = ctypes.c_int64()
        _check(self._lib.fnlb_read_structure_factor(self._h, rep, field, _dp(a2), _dp(re),
                                                    _dp(im), ctypes.byref(n)),
               "fnlb_read_structure_factor")
        return a2, re, im, int(n.value)

    def structure_factor(self, rep: int = 0, field: int = FIELD_C) -> np.ndarray:
        """S(q) = mean |Phi|^2 - |mean Phi|^2, shape [Lz][Lx//2+1]."""
        a2, re, im, n = self.read_structure_factor(rep, field)
        n = max(n, 1)
        return a2 / n - ((re / n) ** 2 + (im / n) ** 2)

    def read_pressure(self, rep: int = 0):
        r = self.reps[rep]
        s, s2 = ctypes.c_double(), ctypes.c_double()
        prof = np.empty(r.Lz)
        n = ctypes.c_int64()
        _check(self._lib.fnlb_read_pressure(self._h, rep, ctypes.byref(s), ctypes.byref(s2),
                                            _dp(prof), ctypes.byref(n)), "fnlb_read_pressure")
        return s.value, s2.value, prof, int(n.value)

    def read_populations(self, rep: int = 0) -> np.ndarray:
        r = self.reps[rep]
        out = np.empty((2, 9, r.Lz, r.Lx))
        _check(self._lib.fnlb_read_populations(self._h, rep, _dp(out)), "fnlb_read_populations")
        return out

    def write_populations(self, rep: int, f: np.ndarray) -> None:
        f = np.ascontiguousarray(f, dtype=np.float64)
        r = self.reps[rep]
        if f.shape != (2, 9, r.Lz, r.Lx):
            raise ValueError(f"populations of shape {f.shape}, expected {(2, 9, r.Lz, r.Lx)}")
        _check(self._lib.fnlb_write_populations(self._h, rep, _dp(f)), "fnlb_write_populations")

    def save(self) -> np.ndarray:
        """Checkpoint image (populations, accumulators, time) as a byte array."""
        nb = ctypes.c_size_t()
        _check(self._lib.fnlb_checkpoint_bytes(self._h, ctypes.byref(nb)),
               "fnlb_checkpoint_bytes")
        buf = np.empty(nb.value, dtype=np.uint8)
        _check(self._lib.fnlb_save(self._h, buf.ctypes.data_as(ctypes.c_void_p), nb.value),
               "fnlb_save")
        return buf

    def load(self, image: np.ndarray) -> None:
        """Restores a checkpoint image made by a handle of the same replicas."""
        buf = np.ascontiguousarray(image, dtype=np.uint8)
        _check(self._lib.fnlb_load(self._h, buf.ctypes.data_as(ctypes.c_void_p), buf.size),
               "fnlb_load")

    def reset_accumulators(self) -> None:
        _check(self._lib.fnlb_reset_accumulators(self._h), "fnlb_reset_accumulators")

    @property
    def time(self) -> int:
        t = ctypes.c_int64()
        _check(self._lib.fnlb_get_time(self._h, ctypes.byref(t)), "fnlb_get_time")
        return int(t.value)

    @time.setter
    def time(self, t: int) -> None:
        _check(self._lib.fnlb_set_time(self._h, int(t)), "fnlb_set_time")


def sq_misfit(theta, rep, S_target, weight, horizon: int, sample_every: int,
              ckpt_every: int = 100, field: int = FIELD_C, device: str = "cuda:0"):
    """Differentiable structure-factor misfit: theta = tensor([tau_s, tau_d, G]).
    Forward runs the step from the rest state on the imposed profile and
    returns J (one forward sweep, on a handle reused across calls); backward
    runs the adjoint sweep over that forward sweep's checkpoints (noise held
    fixed)."""
    return _SqMisfit.apply(theta, rep, S_target, weight, horizon, sample_every, ckpt_every,
                           field, device, "sq")


def p_misfit(theta, rep, P_target, weight, horizon: int, sample_every: int,
             ckpt_every: int = 100, device: str = "cuda:0"):
    """Differentiable pressure-profile misfit: theta = tensor([tau_s, tau_d, G]).
    Forward runs the step from the rest state on the imposed profile and
    returns J (one forward sweep, on a handle reused across calls); backward
    runs the adjoint sweep over that forward sweep's checkpoints (noise held
    fixed)."""
    return _SqMisfit.apply(theta, rep, P_target, weight, horizon, sample_every, ckpt_every,
                           FIELD_C, device, "p")


_MISFIT_LATTICES = {}


def _misfit_lattice(rep, sample_every: int, device: str) -> "Lattice":
    """One handle per (shape, sampling interval, device), reused by the
    differentiable misfits through fnlb_reinit."""
    key = (rep.Lx, rep.Lz, int(sample_every), str(device))
    lat = _MISFIT_LATTICES.get(key)
    if lat is None:
        lat = Lattice([rep], precision=FP64, sample_every=sample_every, device=device)
        _MISFIT_LATTICES[key] = lat
    else:
        lat.reinit([rep])
    return lat


def _make_fn():
    import dataclasses

    import torch

    def forward_sweep(lat, kind, target, weight, horizon, ckpt_every, field):
        if kind == "p":
            return lat.pressure_misfit(target, weight, horizon, ckpt_every)
        return lat.sq_misfit(target, weight, horizon, ckpt_every, field)

    class SqMisfit(torch.autograd.Function):
        @staticmethod
        def forward(ctx, theta, rep, target, weight, horizon, sample_every, ckpt_every,
                    field, device, kind):
            t = [float(v) for v in theta.detach().cpu().tolist()]
            r = dataclasses.replace(rep, tau_s=t[0], tau_d=t[1], G=t[2])
            lat = _misfit_lattice(r, sample_every, device)
            J = forward_sweep(lat, kind, target, weight, horizon, ckpt_every, field)
            ctx.lat, ctx.token = lat, lat._misfit_token
            ctx.redo = (r, kind, target, weight, horizon, ckpt_every, field)
            ctx.theta_dtype = theta.dtype
            return theta.new_tensor(J)

        @staticmethod
        def backward(ctx, gJ):
            lat = ctx.lat
            if lat._misfit_token != ctx.token:
                # the handle has served another evaluation since this forward
                # sweep: run it again before differentiating it
                r, kind, target, weight, horizon, ckpt_every, field = ctx.redo
                lat.reinit([r])
                forward_sweep(lat, kind, target, weight, horizon, ckpt_every, field)
                ctx.token = lat._misfit_token
            g = torch.as_tensor(lat.misfit_backward(), dtype=ctx.theta_dtype)
            return ((gJ.cpu() * g).to(gJ.device), None, None, None, None, None, None, None, None,
                    None)

    return SqMisfit


class _Lazy:
    fn = None

    def apply(self, *a):
        if _Lazy.fn is None:
            _Lazy.fn = _make_fn()
        return _Lazy.fn.apply(*a)


_SqMisfit = _Lazy()
