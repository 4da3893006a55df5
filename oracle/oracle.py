"""ctypes wrapper of the FP64 CPU oracle (fnlb_oracle.cpp).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the GPU library.  All arrays are
numpy float64 in the oracle's own layouts:
  f     [2 species][9 links][Lz][Lx]
  sq    [fields][3 (sum |Phi|^2, sum Re, sum Im)][Lz][Lx//2+1]; fields are
        (delta c, delta rho), plus (U_x, U_z) when VELOCITY is set
  pr    [2] = (sum of spatial means of P - P_ref, sum of their squares)
  prof  [Lz] = sum of row means of P - P_ref
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fnlb_oracle.cpp")
_LIB = os.path.join(_HERE, "libfnlb_oracle.so")

ASTAR, WALL_UZ_FIX, NOISE_LOC, FORCE_LITERAL, VELOCITY = 1, 2, 4, 8, 32
DEFAULT_FLAGS = ASTAR | WALL_UZ_FIX


def build(force: bool = False) -> str:
    """Compile the oracle with g++ -O2 (plain C++, OpenMP over nodes)."""
    stale = (not os.path.exists(_LIB)) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)
    if force or stale:
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC",
                               "-shared", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


class OraParams(ctypes.Structure):
    _fields_ = [("Lx", ctypes.c_int32), ("Lz", ctypes.c_int32),
                ("rho0", ctypes.c_double), ("grad_c0", ctypes.c_double),
                ("kT", ctypes.c_double), ("G", ctypes.c_double),
                ("tau_d", ctypes.c_double), ("tau_s", ctypes.c_double),
                ("tau_e", ctypes.c_double), ("tau_q", ctypes.c_double),
                ("tau_eps", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("flags", ctypes.c_int32), ("sample_every", ctypes.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        dp = ctypes.POINTER(ctypes.c_double)
        pp = ctypes.POINTER(OraParams)
        i64p = ctypes.POINTER(ctypes.c_int64)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        _lib.ora_init.argtypes = [pp, dp]
        _lib.ora_run.argtypes = [pp, ctypes.c_int64, ctypes.c_int64, dp, dp, dp, dp, i64p]
        _lib.ora_sample.argtypes = [pp, dp, dp, dp, dp, i64p]
        _lib.ora_fields.argtypes = [pp, dp, dp, dp]
        _lib.ora_philox4x32_10.argtypes = [u32p, u32p, u32p]
        _lib.ora_node_gaussians.argtypes = [ctypes.c_uint64, ctypes.c_uint32,
                                            ctypes.c_uint64, dp]
        _lib.ora_tables.argtypes = [dp, dp, dp, dp]
        _lib.ora_equilibrium.argtypes = [ctypes.c_double] * 3 + [dp]
        _lib.ora_forcing_moments.argtypes = [ctypes.c_double] * 4 + [dp]
        _lib.ora_check_params.argtypes = [pp]
        _lib.ora_set_num_threads.argtypes = [ctypes.c_int]
        _lib.ora_num_threads.restype = ctypes.c_int
    return _lib


def _dp(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def params(rep, flags: int = DEFAULT_FLAGS, sample_every: int = 0) -> OraParams:
    return OraParams(rep.Lx, rep.Lz, rep.rho0, rep.grad_c0, rep.kT, rep.G,
                     rep.tau_d, rep.tau_s, rep.tau_e, rep.tau_q, rep.tau_eps,
                     rep.seed & ((1 << 64) - 1), flags, sample_every)


class Accum:
    """Oracle-side accumulators for one lattice."""

    def __init__(self, Lx: int, Lz: int, nfields: int = 2):
        self.sq = np.zeros((nfields, 3, Lz, Lx // 2 + 1))
        self.pr = np.zeros(2)
        self.prof = np.zeros(Lz)
        self.n = ctypes.c_int64(0)

    @property
    def n_samples(self) -> int:
        return int(self.n.value)


def set_threads(n: int) -> None:
    lib().ora_set_num_threads(int(n))


def num_threads() -> int:
    return int(lib().ora_num_threads())


def init_state(rep, flags: int = DEFAULT_FLAGS) -> np.ndarray:
    p = params(rep, flags)
    f = np.zeros((2, 9, rep.Lz, rep.Lx))
    if lib().ora_init(ctypes.byref(p), _dp(f)) != 0:
        raise ValueError("oracle: invalid parameters")
    return f


def run(rep, f: np.ndarray, t0: int, nsteps: int, acc: Accum | None = None,
        flags: int = DEFAULT_FLAGS, sample_every: int = 0) -> np.ndarray:
    """Advance f in place from time t0 by nsteps steps; returns f."""
    p = params(rep, flags, sample_every)
    if acc is None:
        rc = lib().ora_run(ctypes.byref(p), t0, nsteps, _dp(f), None, None, None, None)
    else:
        rc = lib().ora_run(ctypes.byref(p), t0, nsteps, _dp(f), _dp(acc.sq),
                           _dp(acc.pr), _dp(acc.prof), ctypes.byref(acc.n))
    if rc != 0:
        raise ValueError("oracle: invalid parameters")
    return f


def sample(rep, f: np.ndarray, acc: Accum, flags: int = DEFAULT_FLAGS) -> None:
    p = params(rep, flags)
    if lib().ora_sample(ctypes.byref(p), _dp(f), _dp(acc.sq), _dp(acc.pr),
                        _dp(acc.prof), ctypes.byref(acc.n)) != 0:
        raise ValueError("oracle: invalid parameters")


def fields(rep, f: np.ndarray, flags: int = DEFAULT_FLAGS):
    """Returns (rho[2][Lz][Lx], dphi[nf][Lz][Lx]) of the state f, nf = 4 with
    VELOCITY in flags (delta c, delta rho, U_x, U_z), else 2."""
    p = params(rep, flags)
    rho = np.zeros((2, rep.Lz, rep.Lx))
    dphi = np.zeros((4 if flags & VELOCITY else 2, rep.Lz, rep.Lx))
    if lib().ora_fields(ctypes.byref(p), _dp(f), _dp(rho), _dp(dphi)) != 0:
        raise ValueError("oracle: invalid parameters")
    return rho, dphi


def check_params(rep) -> bool:
    p = params(rep)
    return lib().ora_check_params(ctypes.byref(p)) == 0


def philox(ctr, key):
    c = (ctypes.c_uint32 * 4)(*ctr)
    k = (ctypes.c_uint32 * 2)(*key)
    o = (ctypes.c_uint32 * 4)()
    lib().ora_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def node_gaussians(seed: int, node: int, t: int) -> np.ndarray:
    g = np.zeros(14)
    lib().ora_node_gaussians(seed, node, t, _dp(g))
    return g


def tables():
    c = np.zeros((9, 2))
    w = np.zeros(9)
    T = np.zeros((9, 9))
    N = np.zeros(9)
    lib().ora_tables(_dp(c), _dp(w), _dp(T), _dp(N))
    return c.astype(int), w, T, N


def equilibrium(rho: float, ux: float, uz: float) -> np.ndarray:
    f = np.zeros(9)
    lib().ora_equilibrium(rho, ux, uz, _dp(f))
    return f


def forcing_moments(ux: float, uz: float, fx: float, fz: float) -> np.ndarray:
    S = np.zeros(9)
    lib().ora_forcing_moments(ux, uz, fx, fz, _dp(S))
    return S


def structure_factor(acc: Accum) -> np.ndarray:
    """S = mean |Phi|^2 - |mean Phi|^2 per field, shape [nf][Lz][Lx//2+1]."""
    n = max(acc.n_samples, 1)
    m2 = acc.sq[:, 0] / n
    mr = acc.sq[:, 1] / n
    mi = acc.sq[:, 2] / n
    return m2 - (mr * mr + mi * mi)


def velocity(rep, f: np.ndarray, flags: int = DEFAULT_FLAGS) -> np.ndarray:
    """Barycentric velocity U[2][Lz][Lx] (after the wall fix) of the state f."""
    p = params(rep, flags)
    U = np.zeros((2, rep.Lz, rep.Lx))
    lib().ora_velocity.argtypes = [ctypes.POINTER(OraParams),
                                   ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(ctypes.c_double)]
    if lib().ora_velocity(ctypes.byref(p), _dp(f), _dp(U)) != 0:
        raise ValueError("oracle: invalid parameters")
    return U


def macros(rep, f: np.ndarray, flags: int = DEFAULT_FLAGS):
    """(fl, F, U) of the state f as the collision uses them: populations after
    the wall fix fl[2][9][Lz][Lx], force densities F[species][component][Lz][Lx]
    and barycentric velocity U[component][Lz][Lx]."""
    p = params(rep, flags)
    fl = np.zeros_like(f)
    F = np.zeros((2, 2, rep.Lz, rep.Lx))
    U = np.zeros((2, rep.Lz, rep.Lx))
    dp = ctypes.POINTER(ctypes.c_double)
    lib().ora_macros.argtypes = [ctypes.POINTER(OraParams), dp, dp, dp, dp]
    if lib().ora_macros(ctypes.byref(p), _dp(f), _dp(fl), _dp(F), _dp(U)) != 0:
        raise ValueError("oracle: invalid parameters")
    return fl, F, U


def _misfit_argtypes():
    dp = ctypes.POINTER(ctypes.c_double)
    pp = ctypes.POINTER(OraParams)
    lib().ora_sq_misfit.argtypes = [pp, ctypes.c_int64, ctypes.c_int, dp, dp, dp]
    lib().ora_sq_misfit_cs.argtypes = [pp, ctypes.c_int64, ctypes.c_int, dp, dp, ctypes.c_int,
                                       ctypes.c_double, dp]


def sq_misfit(rep, horizon: int, every: int, field: int, S_target: np.ndarray,
              weight: np.ndarray, flags: int = DEFAULT_FLAGS) -> float:
    """J = sum_q weight_q (S(q) - S_target(q))^2 over a run of `horizon` steps
    from the rest state, sampled every `every` steps (half spectrum [kz][kx])."""
    _misfit_argtypes()
    p = params(rep, flags, every)
    St = np.ascontiguousarray(S_target, dtype=np.float64)
    w = np.ascontiguousarray(weight, dtype=np.float64)
    J = ctypes.c_double()
    if lib().ora_sq_misfit(ctypes.byref(p), horizon, field, _dp(St), _dp(w), ctypes.byref(J)):
        raise ValueError("oracle: invalid arguments")
    return J.value


def sq_misfit_complex_step(rep, horizon: int, every: int, field: int, S_target: np.ndarray,
                           weight: np.ndarray, which: int, h: float = 1e-20,
                           flags: int = DEFAULT_FLAGS) -> float:
    """dJ/d(tau_s, tau_d, G)[which] by complex-step differentiation of the
    oracle (the simulation templated on std::complex<double>)."""
    _misfit_argtypes()
    p = params(rep, flags, every)
    St = np.ascontiguousarray(S_target, dtype=np.float64)
    w = np.ascontiguousarray(weight, dtype=np.float64)
    d = ctypes.c_double()
    if lib().ora_sq_misfit_cs(ctypes.byref(p), horizon, field, _dp(St), _dp(w), which, h,
                              ctypes.byref(d)):
        raise ValueError("oracle: invalid arguments")
    return d.value


def _p_misfit_argtypes():
    dp = ctypes.POINTER(ctypes.c_double)
    pp = ctypes.POINTER(OraParams)
    lib().ora_p_misfit.argtypes = [pp, ctypes.c_int64, dp, dp, dp]
    lib().ora_p_misfit_cs.argtypes = [pp, ctypes.c_int64, dp, dp, ctypes.c_int, ctypes.c_double,
                                      dp]


def p_misfit(rep, horizon: int, every: int, P_target: np.ndarray, weight: np.ndarray,
             flags: int = DEFAULT_FLAGS) -> float:
    """J = sum_j weight_j (Pbar_j - P_target_j)^2, Pbar_j the time-averaged row
    means of P - P_ref over a run of `horizon` steps sampled every `every`."""
    _p_misfit_argtypes()
    p = params(rep, flags, every)
    Pt = np.ascontiguousarray(P_target, dtype=np.float64)
    w = np.ascontiguousarray(weight, dtype=np.float64)
    J = ctypes.c_double()
    if lib().ora_p_misfit(ctypes.byref(p), horizon, _dp(Pt), _dp(w), ctypes.byref(J)):
        raise ValueError("oracle: invalid arguments")
    return J.value


def p_misfit_complex_step(rep, horizon: int, every: int, P_target: np.ndarray,
                          weight: np.ndarray, which: int, h: float = 1e-20,
                          flags: int = DEFAULT_FLAGS) -> float:
    """dJ/d(tau_s, tau_d, G)[which] of the pressure-profile misfit by
    complex-step differentiation of the oracle."""
    _p_misfit_argtypes()
    p = params(rep, flags, every)
    Pt = np.ascontiguousarray(P_target, dtype=np.float64)
    w = np.ascontiguousarray(weight, dtype=np.float64)
    d = ctypes.c_double()
    if lib().ora_p_misfit_cs(ctypes.byref(p), horizon, _dp(Pt), _dp(w), which, h,
                             ctypes.byref(d)):
        raise ValueError("oracle: invalid arguments")
    return d.value
