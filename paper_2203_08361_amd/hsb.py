"""Python binding of libhsb (include/hsb.h): argument marshalling only.

Every step of the computation runs in the HIP library; this module converts
numpy arrays / torch device tensors to pointers and back.  There is no CPU
fallback: if libhsb.so is missing or the device is not usable, calls raise.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import sys
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhsb.so")

HSB_BSB, HSB_DSB = 0, 1
HSB_OK, HSB_EINVAL, HSB_ENOMEM, HSB_EDEVICE, HSB_ENUMERIC, HSB_EUNSUPPORTED = 0, -1, -2, -3, -4, -6
HSB_ECANCELED = -5
HSB_OPT_INIT_AMP, HSB_OPT_ENERGY_INTERVAL, HSB_OPT_RETURN_BEST, HSB_OPT_PRECISION = 0, 1, 2, 3
HSB_OPT_TIMING, HSB_OPT_KERNEL_MS, HSB_OPT_KERNEL_LAUNCHES, HSB_OPT_LAST_PLAN = 4, 5, 6, 7
HSB_OPT_LOCAL_EXCHANGE = 8
HSB_OPT_GRAPH = 9
HSB_OPT_GRAPH_LAUNCHES = 10
HSB_OPT_AUTOTUNE, HSB_OPT_TILE, HSB_OPT_LAST_TILE = 11, 12, 13
HSB_OPT_CANCELLABLE = 14
HSB_PLAN_FP32, HSB_PLAN_FP4, HSB_PLAN_DIGITS, HSB_PLAN_INCREMENTAL = 0, 1, 2, 3
PLAN_NAMES = {HSB_PLAN_FP32: "fp32", HSB_PLAN_FP4: "fp4", HSB_PLAN_DIGITS: "digits",
              HSB_PLAN_INCREMENTAL: "incremental"}
HSB_PREC_AUTO, HSB_PREC_FP32, HSB_PREC_MIXED, HSB_PREC_DIGITS = 0, 1, 2, 3
HSB_PREC_INCREMENTAL = 4
HSB_THERMO_HEAT, HSB_THERMO_NOSE_HOOVER = 0, 1
HSB_SCHED_QUEUE, HSB_SCHED_CLASSES = 0, 1

EXPORTED = ("hsb_create", "hsb_destroy", "hsb_last_error", "hsb_set_option", "hsb_get_option",
            "hsb_run", "hsb_run_ex", "hsb_plan_info", "hsb_run_batch", "hsb_num_samples",
            "hsb_run_ex_noalloc", "hsb_cancel")
HSB_NOALLOC_SCRATCH_BYTES = 64 << 20

_lib = None


class HSBError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libhsb error {code}: {msg}")
        self.code = code


class hsb_run_args(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_size_t),
        ("variant", ctypes.c_int32), ("steps", ctypes.c_int32), ("R", ctypes.c_int32),
        ("start_step", ctypes.c_int32), ("schedule_steps", ctypes.c_int32),
        ("thermostat", ctypes.c_int32),
        ("a0", ctypes.c_float), ("c0", ctypes.c_float), ("dt", ctypes.c_float),
        ("gamma", ctypes.c_float),
        ("seed", ctypes.c_uint64),
        ("gamma_rep", ctypes.c_void_p), ("x0", ctypes.c_void_p), ("y0", ctypes.c_void_p),
        ("x_out", ctypes.c_void_p), ("y_out", ctypes.c_void_p),
        ("spins", ctypes.c_void_p), ("energy", ctypes.c_void_p),
        ("best_energy", ctypes.c_void_p), ("final_energy", ctypes.c_void_p),
        ("best_step", ctypes.c_void_p),
        ("stream", ctypes.c_void_p),
        ("trace_energy", ctypes.c_void_p), ("trace_tinst", ctypes.c_void_p),
        ("nh_inv_mass", ctypes.c_double), ("nh_temperature", ctypes.c_double),
        ("xi0", ctypes.c_void_p), ("xi_out", ctypes.c_void_p),
        ("stop_step", ctypes.c_void_p),
    ]


class hsb_job(ctypes.Structure):
    _fields_ = [
        ("instance", ctypes.c_int32), ("R", ctypes.c_int32),
        ("c0", ctypes.c_float), ("gamma", ctypes.c_float),
        ("seed", ctypes.c_uint64),
        ("spins", ctypes.c_void_p), ("energy", ctypes.c_void_p),
    ]


class hsb_batch_args(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_size_t),
        ("variant", ctypes.c_int32), ("steps", ctypes.c_int32),
        ("a0", ctypes.c_float), ("dt", ctypes.c_float),
        ("init_amp", ctypes.c_double),
        ("energy_interval", ctypes.c_int32), ("return_best", ctypes.c_int32),
        ("stream", ctypes.c_void_p), ("scheduler", ctypes.c_int32),
    ]


def load_library():
    """Load libhsb.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build() first")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, f32, f64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_float, ctypes.c_double
    L.hsb_create.restype = i32
    L.hsb_create.argtypes = [vp, i32, ctypes.POINTER(vp)]
    L.hsb_destroy.restype = None
    L.hsb_destroy.argtypes = [vp]
    L.hsb_last_error.restype = ctypes.c_char_p
    L.hsb_last_error.argtypes = []
    L.hsb_set_option.restype = i32
    L.hsb_set_option.argtypes = [vp, i32, f64]
    L.hsb_get_option.restype = i32
    L.hsb_get_option.argtypes = [vp, i32, ctypes.POINTER(f64)]
    L.hsb_run.restype = i32
    L.hsb_run.argtypes = [vp, i32, f32, f32, f32, f32, i32, i32, ctypes.c_uint64, vp, vp]
    L.hsb_run_ex.restype = i32
    L.hsb_run_ex.argtypes = [vp, ctypes.POINTER(hsb_run_args)]
    L.hsb_cancel.restype = i32
    L.hsb_cancel.argtypes = [vp]
    L.hsb_run_ex_noalloc.restype = i32
    L.hsb_run_ex_noalloc.argtypes = [vp, ctypes.POINTER(hsb_run_args)]
    L.hsb_plan_info.restype = i32
    L.hsb_plan_info.argtypes = [vp, i32, ctypes.POINTER(i32)]
    L.hsb_num_samples.restype = i32
    L.hsb_num_samples.argtypes = [vp, i32, i32, ctypes.POINTER(i32)]
    L.hsb_run_batch.restype = i32
    L.hsb_run_batch.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(hsb_job), i32,
                                ctypes.POINTER(hsb_batch_args)]
    _lib = L
    return L


def hsb_last_error() -> str:
    return load_library().hsb_last_error().decode()


def _check(rc: int, allow=()):
    if rc != HSB_OK and rc not in allow:
        raise HSBError(rc, hsb_last_error())
    return rc


def hsb_create(J) -> ctypes.c_void_p:
    J = np.ascontiguousarray(J, dtype=np.float32)
    if J.ndim != 2 or J.shape[0] != J.shape[1]:
        raise ValueError("J must be a square matrix")
    h = ctypes.c_void_p()
    _check(load_library().hsb_create(J.ctypes.data, J.shape[0], ctypes.byref(h)))
    return h


def hsb_destroy(h) -> None:
    load_library().hsb_destroy(h)


def hsb_set_option(h, key: int, value: float) -> None:
    _check(load_library().hsb_set_option(h, key, float(value)))


def hsb_get_option(h, key: int) -> float:
    v = ctypes.c_double()
    _check(load_library().hsb_get_option(h, key, ctypes.byref(v)))
    return v.value


def hsb_plan_info(h, variant: int) -> int:
    p = ctypes.c_int()
    _check(load_library().hsb_plan_info(h, variant, ctypes.byref(p)))
    return p.value


def hsb_cancel(h) -> None:
    """Ask the run in progress on h (or its next run) to stop at a sample point."""
    _check(load_library().hsb_cancel(h))


def hsb_run(h, variant, a0, c0, dt, gamma, steps, R, seed, allow_numeric=False):
    """Host-output run: returns (spins int8 [R][N], energy float64 [R], status)."""
    N = _ctx_n(h)
    spins = np.empty((R, N), dtype=np.int8)
    energy = np.empty(R, dtype=np.float64)
    rc = load_library().hsb_run(h, variant, a0, c0, dt, gamma, steps, R, seed & (2**64 - 1),
                                spins.ctypes.data, energy.ctypes.data)
    _check(rc, (HSB_ENUMERIC,) if allow_numeric else ())
    return spins, energy, rc


_sizes = {}


def _ctx_n(h) -> int:
    return _sizes[h.value]


def hsb_num_samples(h, start_step: int, steps: int) -> int:
    n = ctypes.c_int()
    _check(load_library().hsb_num_samples(h, start_step, steps, ctypes.byref(n)))
    return n.value


def hsb_run_ex(h, variant, steps, R, a0, c0, dt, gamma=0.0, seed=0, gamma_rep=None, x0=None,
               y0=None, start_step=0, schedule_steps=0, want_state=False, stream=None,
               allow_numeric=False, out=None, traces=False, nose_hoover=None, xi0=None,
               noalloc=False, allow_cancel=False):
    """Device run through hsb_run_ex.  Tensors are torch CUDA tensors.

    Returns a dict of device tensors: spins [R][N] int8, energy/best_energy/
    final_energy [R] float64, best_step [R] int32, x/y [R][N] float32 when
    want_state, and trace_energy/trace_tinst [n_samples][R] float64 (energy
    and T_inst of eq. (9) at every sample point) when traces.  `out` may pass
    preallocated tensors under the same keys.

    nose_hoover=(inv_mass, T) runs the thermostat of eqs. (6)-(8) in place of
    the constant heating rate (xi starts at -gamma, or at xi0 [R] float64);
    the result then has xi [R] float64, its value after the last step.

    noalloc=True calls hsb_run_ex_noalloc instead (the library allocates no
    device memory for the run; pass preallocated outputs in `out` to keep
    this call itself free of allocations).

    With allow_cancel (or a stop_step tensor in `out`) the result also has
    stop_step [R] int32: the step each replica reached.  A run stopped by
    hsb_cancel raises HSBError(HSB_ECANCELED) unless allow_cancel, in which
    case its outputs are returned with status HSB_ECANCELED.
    """
    import torch

    N = _ctx_n(h)
    dev = torch.device("cuda", torch.cuda.current_device())
    o = dict(out) if out else {}
    o.setdefault("spins", torch.empty((R, N), dtype=torch.int8, device=dev))
    for k in ("energy", "best_energy", "final_energy"):
        o.setdefault(k, torch.empty(R, dtype=torch.float64, device=dev))
    o.setdefault("best_step", torch.empty(R, dtype=torch.int32, device=dev))
    if allow_cancel:
        o.setdefault("stop_step", torch.empty(R, dtype=torch.int32, device=dev))
    if want_state:
        o.setdefault("x", torch.empty((R, N), dtype=torch.float32, device=dev))
        o.setdefault("y", torch.empty((R, N), dtype=torch.float32, device=dev))
    if traces:
        ns = hsb_num_samples(h, start_step, steps)
        for k in ("trace_energy", "trace_tinst"):
            o.setdefault(k, torch.empty((ns, R), dtype=torch.float64, device=dev))
            if tuple(o[k].shape) != (ns, R) or o[k].dtype != torch.float64:
                raise ValueError(f"{k} must be a float64 tensor of shape {(ns, R)}")
    a = hsb_run_args()
    a.struct_size = ctypes.sizeof(hsb_run_args)
    a.variant, a.steps, a.R = variant, steps, R
    a.start_step, a.schedule_steps = start_step, schedule_steps
    a.a0, a.c0, a.dt, a.gamma = a0, c0, dt, gamma
    a.seed = seed & (2**64 - 1)
    keep = []

    def dptr(t, dtype, shape):
        if t is None:
            return None
        t = t.to(device=dev, dtype=dtype).contiguous()
        if tuple(t.shape) != shape:
            raise ValueError(f"expected shape {shape}, got {tuple(t.shape)}")
        keep.append(t)
        return t.data_ptr()

    a.gamma_rep = dptr(gamma_rep, torch.float32, (R,))
    if nose_hoover is not None:
        a.thermostat = HSB_THERMO_NOSE_HOOVER
        a.nh_inv_mass, a.nh_temperature = float(nose_hoover[0]), float(nose_hoover[1])
        o.setdefault("xi", torch.empty(R, dtype=torch.float64, device=dev))
        a.xi_out = o["xi"].data_ptr()
        a.xi0 = dptr(xi0, torch.float64, (R,))
    elif xi0 is not None:
        raise ValueError("xi0 needs nose_hoover")
    a.x0 = dptr(x0, torch.float32, (R, N))
    a.y0 = dptr(y0, torch.float32, (R, N))
    a.x_out = o["x"].data_ptr() if want_state else None
    a.y_out = o["y"].data_ptr() if want_state else None
    a.spins = o["spins"].data_ptr()
    a.energy = o["energy"].data_ptr()
    a.best_energy = o["best_energy"].data_ptr()
    a.final_energy = o["final_energy"].data_ptr()
    a.best_step = o["best_step"].data_ptr()
    a.stop_step = o["stop_step"].data_ptr() if "stop_step" in o else None
    if traces:
        a.trace_energy = o["trace_energy"].data_ptr()
        a.trace_tinst = o["trace_tinst"].data_ptr()
    s = stream if stream is not None else torch.cuda.current_stream()
    a.stream = s.cuda_stream
    L = load_library()
    rc = (L.hsb_run_ex_noalloc if noalloc else L.hsb_run_ex)(h, ctypes.byref(a))
    _check(rc, ((HSB_ENUMERIC,) if allow_numeric else ()) + ((HSB_ECANCELED,) if allow_cancel else ()))
    o["status"] = rc
    return o


def hsb_run_batch(contexts, jobs, variant, steps, a0, dt, init_amp=0.1, energy_interval=100,
                  return_best=True, stream=None, allow_numeric=False, scheduler=HSB_SCHED_QUEUE,
                  outs=None):
    """Batch of jobs over several instances (hsb_run_batch).

    contexts: list of Context; jobs: list of dicts with keys instance, R, c0,
    gamma, seed.  Returns (list of {"spins", "energy"} device tensors, status).
    outs may pass the output tensors of an earlier call (the same buffers let
    a repeated batch run as one graph launch).
    """
    import torch

    dev = torch.device("cuda", torch.cuda.current_device())
    hs = (ctypes.c_void_p * len(contexts))(*[c.h.value for c in contexts])
    arr = (hsb_job * max(len(jobs), 1))()
    reuse = outs is not None
    outs = list(outs) if reuse else []
    for k, jd in enumerate(jobs):
        i = jd["instance"]
        N = contexts[i].N if 0 <= i < len(contexts) else 1  # the library rejects bad indices
        R = max(jd["R"], 1)
        if reuse:
            o = outs[k]
        else:
            o = {"spins": torch.empty((R, N), dtype=torch.int8, device=dev),
                 "energy": torch.empty(R, dtype=torch.float64, device=dev)}
            outs.append(o)
        j = arr[k]
        j.instance, j.R, j.c0, j.gamma = jd["instance"], jd["R"], jd["c0"], jd["gamma"]
        j.seed = jd["seed"] & (2**64 - 1)
        j.spins, j.energy = o["spins"].data_ptr(), o["energy"].data_ptr()
    a = hsb_batch_args()
    a.struct_size = ctypes.sizeof(hsb_batch_args)
    a.variant, a.steps, a.a0, a.dt = variant, steps, a0, dt
    a.init_amp, a.energy_interval, a.return_best = init_amp, energy_interval, int(return_best)
    a.scheduler = scheduler
    s = stream if stream is not None else torch.cuda.current_stream()
    a.stream = s.cuda_stream
    rc = load_library().hsb_run_batch(hs, len(contexts), arr, len(jobs), ctypes.byref(a))
    _check(rc, (HSB_ENUMERIC,) if allow_numeric else ())
    return outs, rc


# Contexts still open; closed by an exit handler that runs before the
# interpreter (and the HIP runtime beneath it) starts tearing down, so that
# hsb_destroy never runs during finalisation.
_live = weakref.WeakSet()
_is_finalizing = sys.is_finalizing


@atexit.register
def _close_all():
    for c in list(_live):
        try:
            c.close()
        except Exception:
            pass


class Context:
    """Owns one hsb_ctx (the J store) and its options."""

    def __init__(self, J, **options):
        J = np.ascontiguousarray(J, dtype=np.float32)
        self.N = J.shape[0]
        self.h = None
        self.h = hsb_create(J)
        _sizes[self.h.value] = self.N
        _live.add(self)
        for k, v in options.items():
            self.set_option(k, v)

    _KEYS = {"init_amp": HSB_OPT_INIT_AMP, "energy_interval": HSB_OPT_ENERGY_INTERVAL,
             "return_best": HSB_OPT_RETURN_BEST, "precision": HSB_OPT_PRECISION,
             "timing": HSB_OPT_TIMING, "kernel_ms": HSB_OPT_KERNEL_MS,
             "kernel_launches": HSB_OPT_KERNEL_LAUNCHES, "last_plan": HSB_OPT_LAST_PLAN,
             "local_exchange": HSB_OPT_LOCAL_EXCHANGE, "graph": HSB_OPT_GRAPH,
             "graph_launches": HSB_OPT_GRAPH_LAUNCHES, "autotune": HSB_OPT_AUTOTUNE,
             "tile": HSB_OPT_TILE, "last_tile": HSB_OPT_LAST_TILE,
             "cancellable": HSB_OPT_CANCELLABLE}
    _PREC = {"auto": HSB_PREC_AUTO, "fp32": HSB_PREC_FP32, "mixed": HSB_PREC_MIXED,
             "digits": HSB_PREC_DIGITS, "incremental": HSB_PREC_INCREMENTAL}

    def set_option(self, key, value):
        if isinstance(value, str):
            value = self._PREC[value]
        hsb_set_option(self.h, self._KEYS.get(key, key), value)

    def get_option(self, key):
        return hsb_get_option(self.h, self._KEYS.get(key, key))

    def plan(self, variant):
        return {HSB_PREC_FP32: "fp32", HSB_PREC_MIXED: "mixed",
                HSB_PREC_INCREMENTAL: "incremental"}[hsb_plan_info(self.h, variant)]

    def last_plan(self):
        """Execution plan of the last successful run: "fp32", "fp4", "digits" or
        "incremental"."""
        return PLAN_NAMES.get(int(self.get_option("last_plan")))

    def run(self, variant, a0, c0, dt, gamma, steps, R, seed, allow_numeric=False):
        return hsb_run(self.h, variant, a0, c0, dt, gamma, steps, R, seed, allow_numeric)

    def cancel(self):
        """hsb_cancel: stop the run in progress (or the next one) at a sample point."""
        hsb_cancel(self.h)

    def num_samples(self, start_step, steps):
        return hsb_num_samples(self.h, start_step, steps)

    def run_ex(self, variant, steps, R, a0, c0, dt, gamma=0.0, seed=0, **kw):
        return hsb_run_ex(self.h, variant, steps, R, a0, c0, dt, gamma, seed, **kw)

    def close(self):
        """Destroy the context now (its device memory, streams and graphs)."""
        h, self.h = self.h, None
        _live.discard(self)
        if h is not None and h.value:
            _sizes.pop(h.value, None)
            hsb_destroy(h)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        # during interpreter shutdown the runtime below may already be gone
        # (and this module's globals cleared): contexts are closed by the exit
        # handler before that, never here
        try:
            if self.h is None or _is_finalizing():
                return
            self.close()
        except Exception:
            pass
