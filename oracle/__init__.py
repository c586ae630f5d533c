"""CPU oracle for heated simulated bifurcation -- TEST INFRASTRUCTURE ONLY.

A plain, slow C implementation (``hsb_oracle.c``) of what the GPU library
computes, reached through ctypes.  Only the test suite, the smoke check and
the benchmark's CPU-baseline leg use it; the GPU library never does, and the
two share no code.  See ``hsb_oracle.c`` for the passages of the paper each
function follows.

Parity pins (what fixes each function independently of this code) are in
``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hsb_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libhsb_oracle.so")
_lib = None

BSB, DSB = 0, 1
FP64, FP32 = 0, 1


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no GPU toolchain involved)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
               "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Params(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("R", ctypes.c_int32), ("steps", ctypes.c_int32),
                ("variant", ctypes.c_int32), ("interval", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("return_best", ctypes.c_int32),
                ("start_step", ctypes.c_int32), ("schedule_steps", ctypes.c_int32),
                ("thermostat", ctypes.c_int32),
                ("a0", ctypes.c_double), ("c0", ctypes.c_double), ("dt", ctypes.c_double),
                ("gamma", ctypes.c_double), ("gamma_rep", ctypes.c_void_p),
                ("nh_inv_mass", ctypes.c_double), ("nh_temperature", ctypes.c_double),
                ("xi0", ctypes.c_void_p)]


class _Outputs(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in
                ("x", "y", "spins", "energy", "best_e", "final_e", "best_step", "trace_e",
                 "trace_tinst", "xi")]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        vp, i32, u64, f32, f64 = (ctypes.c_void_p, ctypes.c_int, ctypes.c_uint64,
                                  ctypes.c_float, ctypes.c_double)
        L.orc_key.restype = u64
        L.orc_key.argtypes = [u64, u64, u64, u64]
        L.orc_uniform_open.restype = f32
        L.orc_uniform_open.argtypes = [u64, u64, u64, u64]
        L.orc_init_state.restype = None
        L.orc_init_state.argtypes = [u64, i32, i32, i32, f32, vp, vp]
        L.orc_energy.restype = f64
        L.orc_energy.argtypes = [i32, vp, vp]
        L.orc_cut.restype = f64
        L.orc_cut.argtypes = [i32, vp, vp]
        L.orc_brute_force.restype = f64
        L.orc_brute_force.argtypes = [i32, vp, vp, vp]
        L.orc_field.restype = None
        L.orc_field.argtypes = [i32, vp, vp, i32, vp]
        L.orc_update64.restype = None
        L.orc_update64.argtypes = [i32, vp, f64, f64, f64, f64, f64, vp, vp]
        L.orc_update32.restype = None
        L.orc_update32.argtypes = [i32, vp, f32, f32, f32, f32, f32, vp, vp]
        L.orc_num_samples.restype = i32
        L.orc_num_samples.argtypes = [i32, i32]
        L.orc_num_samples_range.restype = i32
        L.orc_num_samples_range.argtypes = [i32, i32, i32]
        L.orc_run.restype = i32
        L.orc_run.argtypes = [ctypes.POINTER(_Params), vp, vp, vp, ctypes.POINTER(_Outputs)]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _J64(J):
    J = np.ascontiguousarray(J, dtype=np.float64)
    if J.ndim != 2 or J.shape[0] != J.shape[1]:
        raise ValueError("J must be square")
    return J


def key(seed, stream, a, b) -> int:
    return int(lib().orc_key(seed & (2**64 - 1), stream, a, b))


def uniform_open(seed, stream, a, b) -> float:
    return float(lib().orc_uniform_open(seed & (2**64 - 1), stream, a, b))


def init_state(seed: int, R: int, N: int, amp: float = 0.1, r0: int = 0):
    """Initial (x0, y0) as float32 [R][N] for replicas r0 .. r0+R-1."""
    x0 = np.empty((R, N), dtype=np.float32)
    y0 = np.empty((R, N), dtype=np.float32)
    lib().orc_init_state(seed & (2**64 - 1), r0, R, N, amp, _p(x0), _p(y0))
    return x0, y0


def energy(J, s) -> float:
    """Eq. (1) for one spin vector s (+-1)."""
    J = _J64(J)
    s = np.ascontiguousarray(s, dtype=np.int8)
    return float(lib().orc_energy(J.shape[0], _p(J), _p(s)))


def energies(J, S) -> np.ndarray:
    """Eq. (1) for each row of S."""
    return np.array([energy(J, s) for s in np.atleast_2d(S)])


def cut(J, s) -> float:
    """Eq. (13) with w = -J."""
    J = _J64(J)
    s = np.ascontiguousarray(s, dtype=np.int8)
    return float(lib().orc_cut(J.shape[0], _p(J), _p(s)))


def brute_force(J):
    """(E_min, first minimiser, number of minimisers) by exhaustive search."""
    J = _J64(J)
    N = J.shape[0]
    s = np.empty(N, dtype=np.int8)
    n = ctypes.c_longlong(0)
    e = lib().orc_brute_force(N, _p(J), _p(s), ctypes.addressof(n))
    return float(e), s, int(n.value)


def field(J, x, variant: int) -> np.ndarray:
    """Eq. (4) (variant 0) or eq. (5) (variant 1) for one replica, FP64."""
    J = _J64(J)
    x = np.ascontiguousarray(x, dtype=np.float64)
    f = np.empty_like(x)
    lib().orc_field(J.shape[0], _p(J), _p(x), variant, _p(f))
    return f


def update(f, x, y, p, a0, c0, dt, gamma, precision: int = FP64):
    """One application of eqs. (16)-(22) given the field f; returns (x, y) new."""
    N = len(x)
    f = np.ascontiguousarray(f, dtype=np.float64)
    if precision == FP64:
        x = np.array(x, dtype=np.float64)
        y = np.array(y, dtype=np.float64)
        lib().orc_update64(N, _p(f), p, a0, c0, dt, gamma, _p(x), _p(y))
    else:
        x = np.array(x, dtype=np.float32)
        y = np.array(y, dtype=np.float32)
        lib().orc_update32(N, _p(f), p, a0, c0, dt, gamma, _p(x), _p(y))
    return x, y


def num_samples(steps: int, interval: int) -> int:
    return int(lib().orc_num_samples(steps, interval))


def run(J, variant: int, a0: float, c0: float, dt: float, gamma, steps: int, R: int,
        seed: int = 0, amp: float = 0.1, interval: int = 100, precision: int = FP64,
        return_best: bool = True, x0=None, y0=None, r0: int = 0, traces: bool = False,
        start_step: int = 0, schedule_steps: int = 0, nose_hoover=None, xi0=None):
    """Run R replicas (replica ids r0 .. r0+R-1) for `steps` steps.

    nose_hoover=(inv_mass, T) replaces the constant heating rate gamma by the
    thermostat variable xi of eqs. (6)-(8) (rate -xi; xi starts at -gamma or
    at xi0 [R]); the result then has "xi", its value after the last step.

    start_step/schedule_steps resume a run: steps k = start_step .. start_step+steps-1
    of a pump schedule a(t_k) = a0 k / schedule_steps (0 means start_step + steps).

    gamma may be a scalar or a per-replica array of length R.  x0/y0 default to
    the seeded initial state.  Returns a dict of numpy arrays.
    """
    J = _J64(J)
    N = J.shape[0]
    if x0 is None or y0 is None:
        gx, gy = init_state(seed, R, N, amp, r0)
        x0 = gx if x0 is None else x0
        y0 = gy if y0 is None else y0
    x0 = np.ascontiguousarray(x0, dtype=np.float32).reshape(R, N)
    y0 = np.ascontiguousarray(y0, dtype=np.float32).reshape(R, N)
    P = _Params()
    P.N, P.R, P.steps, P.variant = N, R, steps, variant
    P.interval, P.precision, P.return_best = interval, precision, int(bool(return_best))
    P.start_step, P.schedule_steps = start_step, schedule_steps
    P.a0, P.c0, P.dt = a0, c0, dt
    xi_arr = None
    if nose_hoover is not None:
        P.thermostat = 1
        P.nh_inv_mass, P.nh_temperature = float(nose_hoover[0]), float(nose_hoover[1])
        if xi0 is not None:
            xi_arr = np.ascontiguousarray(xi0, dtype=np.float64).reshape(R)
            P.xi0 = xi_arr.ctypes.data
    g_arr = None
    if np.ndim(gamma) == 0:
        P.gamma = float(gamma)
        P.gamma_rep = None
    else:
        g_arr = np.ascontiguousarray(gamma, dtype=np.float64)
        if g_arr.shape != (R,):
            raise ValueError("per-replica gamma must have length R")
        P.gamma = 0.0
        P.gamma_rep = g_arr.ctypes.data
    ns = int(lib().orc_num_samples_range(start_step, start_step + steps, interval))
    out = {
        "x": np.empty((R, N)), "y": np.empty((R, N)),
        "spins": np.empty((R, N), dtype=np.int8), "energy": np.empty(R),
        "best_e": np.empty(R), "final_e": np.empty(R),
        "best_step": np.empty(R, dtype=np.int32),
    }
    if traces:
        out["trace_e"] = np.empty((ns, R))
        out["trace_tinst"] = np.empty((ns, R))
    if nose_hoover is not None:
        out["xi"] = np.empty(R)
    O = _Outputs()
    for name in ("x", "y", "spins", "energy", "best_e", "final_e", "best_step", "trace_e",
                 "trace_tinst", "xi"):
        setattr(O, name, out[name].ctypes.data if name in out else None)
    rc = lib().orc_run(ctypes.byref(P), _p(J), _p(x0), _p(y0), ctypes.byref(O))
    if rc == -1:
        raise ValueError("invalid oracle arguments")
    out["status"] = rc
    return out


def step_to_solution(P: float, Ns: int) -> float:
    """Eq. (15): S = Ns log(0.01) / log(1 - P); inf when P = 0, Ns when P >= 0.99."""
    if P <= 0.0:
        return math.inf
    if P >= 0.99:
        return float(Ns)
    return Ns * math.log(0.01) / math.log(1.0 - P)
