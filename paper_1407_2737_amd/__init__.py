"""Python binding of libmhkmc (include/mhkmc.h): argument marshalling only.

Every step of the kinetic Monte-Carlo path runs in the library's HIP kernels; this
module converts numpy arrays to pointers and return codes to exceptions. Importing it
fails loudly when the built library is missing (build it with
``python -m paper_1407_2737_amd.build``).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmhkmc.so")

FP64, FP32_FIELD, BF16X3_WM = 0, 1, 2
P_TWO_STATE, P_SINGLE_RATE = 0, 1
EXTREMA_EXACT, EXTREMA_SCAN200 = 0, 1
ENOTREADY = -5

SYMBOLS = [
    "mh_ctx_create", "mh_ctx_destroy", "mh_create_assembly", "mh_destroy_assembly",
    "mh_run_loops", "mh_run_batch", "mh_sync", "mh_get_loop", "mh_get_sar",
    "mh_get_replica_areas", "mh_get_moments", "mh_debug_steps", "mh_debug_philox",
    "mh_debug_sw", "mh_debug_field", "mh_strerror", "mh_ctx_set_timing", "mh_ctx_get_timing",
    "mh_server_create", "mh_server_submit", "mh_server_poll", "mh_server_destroy",
    "mh_set_replica_fields", "mh_get_area_per_np", "mh_run_mean_loop",
    "mh_ctx_autotune", "mh_ctx_load_shapes", "mh_get_dhdip",
    "mh_get_local_concentration", "mh_create_assembly_sets", "mh_get_field_error",
    "mh_debug_sw_mode", "mh_field_noalloc", "mh_time_kernels", "mh_time_empty_steps",
]


class MHError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__(f"{what}: {_lib().mh_strerror(code).decode()} ({code})")


class Params(C.Structure):
    _fields_ = [("Ms", C.c_double), ("Keff", C.c_double), ("d", C.c_double), ("T", C.c_double),
                ("tau0", C.c_double), ("rho", C.c_double), ("f", C.c_double),
                ("mu0Hmax", C.c_double), ("dt_override", C.c_double),
                ("field_dir", C.c_double * 3), ("steps_per_period", C.c_int32), ("n_periods", C.c_int32),
                ("n_discard", C.c_int32), ("prob_form", C.c_int32), ("precision", C.c_int32),
                ("interactions", C.c_int32), ("extrema_mode", C.c_int32),
                ("reserved", C.c_int32)]

    @classmethod
    def make(cls, precision: int = FP64, **kw) -> "Params":
        p = cls()
        defaults = dict(Ms=4.0e5, Keff=1.3e4, d=12e-9, T=300.0, tau0=1e-10, rho=5200.0, f=1e5,
                        mu0Hmax=0.02, dt_override=0.0, steps_per_period=2000, n_periods=3,
                        n_discard=2, prob_form=0, interactions=1, extrema_mode=0,
                        field_dir=(1.0, 0.0, 0.0))
        defaults.update({k: v for k, v in kw.items() if k in defaults})
        for k, v in defaults.items():
            setattr(p, k, (C.c_double * 3)(*v) if k == "field_dir" else v)
        p.precision = precision
        return p


class Request(C.Structure):
    _fields_ = [("n", C.c_int64), ("pos", C.POINTER(C.c_double)), ("axes", C.POINTER(C.c_double)),
                ("n_axes_sets", C.c_int64), ("params", Params), ("seed", C.c_uint64),
                ("target_rel_err", C.c_double), ("abs_err_floor", C.c_double),
                ("min_replicas", C.c_int64),
                ("max_replicas", C.c_int64)]


class Result(C.Structure):
    _fields_ = [("sar_Wkg", C.c_double), ("sar_se", C.c_double), ("area_Jm3", C.c_double),
                ("area_se", C.c_double), ("loops", C.c_int64), ("replicas", C.c_int64),
                ("submit_ns", C.c_uint64), ("start_ns", C.c_uint64), ("done_ns", C.c_uint64),
                ("status", C.c_int32)]


_L = None


def _lib():
    global _L
    if _L is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with python -m paper_1407_2737_amd.build")
        L = C.CDLL(LIB_PATH)
        vp, i64, u64, i32, dp = C.c_void_p, C.c_int64, C.c_uint64, C.c_int32, C.POINTER(C.c_double)
        u64p = C.POINTER(C.c_uint64)
        sig = {
            "mh_ctx_create": ([C.c_int, C.POINTER(vp)], C.c_int),
            "mh_ctx_destroy": ([vp], C.c_int),
            "mh_create_assembly": ([vp, i64, dp, dp, i64, C.POINTER(Params), C.POINTER(vp)], C.c_int),
            "mh_create_assembly_sets": ([vp, i64, dp, i64, dp, i64, C.POINTER(Params),
                                         C.POINTER(vp)], C.c_int),
            "mh_destroy_assembly": ([vp], C.c_int),
            "mh_run_loops": ([vp, i64, u64, vp], C.c_int),
            "mh_run_batch": ([C.POINTER(vp), i32, C.POINTER(i64), u64p, vp], C.c_int),
            "mh_time_kernels": ([C.POINTER(vp), i32, i32, i32, i32, dp], C.c_int),
            "mh_time_empty_steps": ([vp, i64, dp], C.c_int),
            "mh_sync": ([vp], C.c_int),
            "mh_get_loop": ([vp, i64, i32, dp, dp], C.c_int),
            "mh_get_sar": ([vp, dp, dp, dp, dp, dp], C.c_int),
            "mh_get_replica_areas": ([vp, dp], C.c_int),
            "mh_get_moments": ([vp, i64, dp], C.c_int),
            "mh_get_area_per_np": ([vp, i64, dp], C.c_int),
            "mh_get_dhdip": ([vp, i64, dp], C.c_int),
            "mh_get_field_error": ([vp, i64, dp, dp], C.c_int),
            "mh_get_local_concentration": ([vp, i32, dp], C.c_int),
            "mh_run_mean_loop": ([vp, i64, vp], C.c_int),
            "mh_ctx_autotune": ([vp, i32, C.POINTER(i64), i32, C.POINTER(i64), i32, C.c_char_p],
                                C.c_int),
            "mh_ctx_load_shapes": ([vp, C.c_char_p], C.c_int),
            "mh_debug_steps": ([vp, i64, u64, i64, i64, dp, dp], C.c_int),
            "mh_debug_philox": ([vp, u64, u64, i64, u64p, u64p], C.c_int),
            "mh_debug_sw": ([vp, i64, dp, dp, dp, dp], C.c_int),
            "mh_debug_sw_mode": ([vp, i32, i64, dp, dp, dp, dp], C.c_int),
            "mh_debug_field": ([vp, dp, dp], C.c_int),
            "mh_field_noalloc": ([vp, vp, vp, vp], C.c_int),
            "mh_strerror": ([C.c_int], C.c_char_p),
            "mh_ctx_set_timing": ([vp, C.c_int], C.c_int),
            "mh_ctx_get_timing": ([vp, i32, dp, C.POINTER(i64)], C.c_int),
            "mh_server_create": ([vp, C.c_size_t, C.POINTER(vp)], C.c_int),
            "mh_server_submit": ([vp, C.POINTER(Request), C.POINTER(u64)], C.c_int),
            "mh_server_poll": ([vp, u64, C.POINTER(Result)], C.c_int),
            "mh_server_destroy": ([vp], C.c_int),
            "mh_set_replica_fields": ([vp, i64, dp], C.c_int),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _L = L
    return _L


def _check(code: int, what: str):
    if code != 0:
        raise MHError(code, what)


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None and a.shape != shape:
        a = a.reshape(shape)
    return a


class Context:
    """A device context (mh_ctx_create)."""

    def __init__(self, device: int = 0):
        self._h = C.c_void_p()
        _check(_lib().mh_ctx_create(device, C.byref(self._h)), "mh_ctx_create")

    def close(self):
        if self._h:
            _lib().mh_ctx_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_timing(self, on: bool):
        _check(_lib().mh_ctx_set_timing(self._h, 1 if on else 0), "mh_ctx_set_timing")

    def time_empty_steps(self, steps: int = 6000) -> float:
        """mh_time_empty_steps: microseconds per empty resident step (one LDS exchange and
        one barrier in one workgroup), the latency floor of a resident step."""
        us = C.c_double()
        _check(_lib().mh_time_empty_steps(self._h, steps, C.byref(us)), "mh_time_empty_steps")
        return us.value

    def get_timing(self, kind: int = 0):
        """(summed ms, launches) of the recorded step-kernel launches of one kind."""
        ms = C.c_double()
        cnt = C.c_int64()
        _check(_lib().mh_ctx_get_timing(self._h, kind, C.byref(ms), C.byref(cnt)),
               "mh_ctx_get_timing")
        return ms.value, cnt.value

    def autotune(self, precision: int, sizes, replicas=(1,), json_path: str | None = None):
        """Time the field-kernel launch shapes (mh_ctx_autotune); sizes=() clears."""
        sz = np.ascontiguousarray(sizes, dtype=np.int64)
        rp = np.ascontiguousarray(replicas, dtype=np.int64)
        p64 = C.POINTER(C.c_int64)
        _check(_lib().mh_ctx_autotune(self._h, precision, sz.ctypes.data_as(p64), sz.shape[0],
                                      rp.ctypes.data_as(p64), rp.shape[0],
                                      json_path.encode() if json_path else None),
               "mh_ctx_autotune")

    def load_shapes(self, json_path: str):
        _check(_lib().mh_ctx_load_shapes(self._h, json_path.encode()), "mh_ctx_load_shapes")

    def debug_philox(self, seed: int, stream: int, ctr: np.ndarray) -> np.ndarray:
        ctr = np.ascontiguousarray(ctr, dtype=np.uint64).reshape(-1, 4)
        out = np.empty_like(ctr)
        p = C.POINTER(C.c_uint64)
        _check(_lib().mh_debug_philox(self._h, seed, stream, ctr.shape[0], ctr.ctypes.data_as(p),
                                      out.ctypes.data_as(p)), "mh_debug_philox")
        return out

    def debug_sw(self, hx, hy, theta0, extrema_mode: int = EXTREMA_EXACT) -> np.ndarray:
        hx, hy, th = _f64(hx).ravel(), _f64(hy).ravel(), _f64(theta0).ravel()
        out = np.empty((hx.shape[0], 6))
        if extrema_mode == EXTREMA_EXACT:
            _check(_lib().mh_debug_sw(self._h, hx.shape[0], _dp(hx), _dp(hy), _dp(th), _dp(out)),
                   "mh_debug_sw")
        else:
            _check(_lib().mh_debug_sw_mode(self._h, extrema_mode, hx.shape[0], _dp(hx), _dp(hy),
                                           _dp(th), _dp(out)), "mh_debug_sw_mode")
        return out


class Assembly:
    """An assembly of particles (mh_create_assembly) and its last run."""

    def __init__(self, ctx: Context, pos, axes, params: Params, n_axes_sets: int = 1,
                 n_pos_sets: int = 1):
        self.ctx = ctx
        pos = _f64(pos)
        self.n = pos.shape[0] // n_pos_sets
        pos = _f64(pos, (n_pos_sets * self.n, 3))
        axes = _f64(axes, (n_axes_sets * self.n, 3))
        self.params = params
        self._h = C.c_void_p()
        if n_pos_sets == 1:
            _check(_lib().mh_create_assembly(ctx._h, self.n, _dp(pos), _dp(axes), n_axes_sets,
                                             C.byref(params), C.byref(self._h)),
                   "mh_create_assembly")
        else:
            _check(_lib().mh_create_assembly_sets(ctx._h, self.n, _dp(pos), n_pos_sets, _dp(axes),
                                                  n_axes_sets, C.byref(params), C.byref(self._h)),
                   "mh_create_assembly_sets")
        self.R = 0

    def close(self):
        if self._h:
            _lib().mh_destroy_assembly(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_replica_fields(self, mu0Hmax):
        """Per-replica field amplitudes (T); replica r uses mu0Hmax[r mod len]."""
        h = _f64(mu0Hmax).ravel()
        _check(_lib().mh_set_replica_fields(self._h, h.shape[0], _dp(h) if h.size else None),
               "mh_set_replica_fields")

    def run(self, n_replicas: int = 1, seed: int = 0, stream=None):
        _check(_lib().mh_run_loops(self._h, n_replicas, seed, stream), "mh_run_loops")
        self.R = n_replicas

    def run_mean_loop(self, n_replicas: int = 1, stream=None):
        """Deterministic mean-magnetisation loops (non-interacting particles)."""
        _check(_lib().mh_run_mean_loop(self._h, n_replicas, stream), "mh_run_mean_loop")
        self.R = n_replicas

    def sync(self):
        _check(_lib().mh_sync(self._h), "mh_sync")

    def loop(self, replica: int = 0, period: int = 0):
        S = self.params.steps_per_period
        H = np.empty(S)
        M = np.empty(S)
        _check(_lib().mh_get_loop(self._h, replica, period, _dp(H), _dp(M)), "mh_get_loop")
        return H, M

    def sar(self, per_np: bool = False):
        v = [C.c_double() for _ in range(4)]
        apn = np.empty(self.n) if per_np else None
        _check(_lib().mh_get_sar(self._h, *[C.byref(x) for x in v],
                                 _dp(apn) if per_np else None), "mh_get_sar")
        out = dict(sar=v[0].value, sar_se=v[1].value, area=v[2].value, area_se=v[3].value)
        if per_np:
            out["area_per_np"] = apn
        return out

    def replica_areas(self) -> np.ndarray:
        out = np.empty(self.R)
        _check(_lib().mh_get_replica_areas(self._h, _dp(out)), "mh_get_replica_areas")
        return out

    def area_per_np(self, replica: int = 0) -> np.ndarray:
        """Per-particle loop areas of one replica, J/m^3 (mean over kept periods)."""
        out = np.empty(self.n)
        _check(_lib().mh_get_area_per_np(self._h, replica, _dp(out)), "mh_get_area_per_np")
        return out

    def local_concentration(self, N: int = 20) -> np.ndarray:
        """Eq. 8 phi_N of every particle."""
        out = np.empty(self.n)
        _check(_lib().mh_get_local_concentration(self._h, N, _dp(out)),
               "mh_get_local_concentration")
        return out

    def field_error(self, replica: int = 0):
        """(relative Frobenius, max over rms) of this form's field against FP64."""
        rel, mx = C.c_double(), C.c_double()
        _check(_lib().mh_get_field_error(self._h, replica, C.byref(rel), C.byref(mx)),
               "mh_get_field_error")
        return rel.value, mx.value

    def dhdip(self, replica: int = 0) -> np.ndarray:
        """Eq. 6 per particle of one replica, tesla (mean over kept periods)."""
        out = np.empty(self.n)
        _check(_lib().mh_get_dhdip(self._h, replica, _dp(out)), "mh_get_dhdip")
        return out

    def moments(self, replica: int = 0) -> np.ndarray:
        out = np.empty((self.n, 3))
        _check(_lib().mh_get_moments(self._h, replica, _dp(out)), "mh_get_moments")
        return out

    def debug_steps(self, n_replicas: int, seed: int, k0: int, k1: int, m_in=None, diag=True):
        m = None if m_in is None else _f64(m_in, (n_replicas * self.n, 3))
        d = np.empty((n_replicas, self.n, 8)) if diag else None
        _check(_lib().mh_debug_steps(self._h, n_replicas, seed, k0, k1,
                                     _dp(m) if m is not None else None,
                                     _dp(d) if d is not None else None), "mh_debug_steps")
        self.R = n_replicas
        return d

    def debug_field(self, m) -> np.ndarray:
        m = _f64(m, (self.n, 3))
        out = np.empty((self.n, 3))
        _check(_lib().mh_debug_field(self._h, _dp(m), _dp(out)), "mh_debug_field")
        return out

    def field_noalloc(self, d_m: int, d_B: int, stream: int | None = None) -> None:
        """mh_field_noalloc: d_m, d_B are device addresses of n x 3 doubles; only
        enqueues kernels on ``stream`` (None: the library's stream)."""
        _check(_lib().mh_field_noalloc(self._h, C.c_void_p(d_m), C.c_void_p(d_B),
                                       C.c_void_p(stream) if stream else None),
               "mh_field_noalloc")


class Server:
    """Continuous-batching server (mh_server_*)."""

    def __init__(self, ctx: Context, hbm_budget_bytes: int):
        self._h = C.c_void_p()
        _check(_lib().mh_server_create(ctx._h, hbm_budget_bytes, C.byref(self._h)),
               "mh_server_create")

    def submit(self, pos, axes, params: Params, seed: int, target_rel_err: float = 0.01,
               min_replicas: int = 64, max_replicas: int = 8192, n_axes_sets: int = 1,
               abs_err_floor: float = 0.0) -> int:
        pos = _f64(pos)
        axes = _f64(axes, (n_axes_sets * pos.shape[0], 3))
        rq = Request(pos.shape[0], _dp(pos), _dp(axes), n_axes_sets, params, seed, target_rel_err,
                     abs_err_floor, min_replicas, max_replicas)
        rid = C.c_uint64()
        _check(_lib().mh_server_submit(self._h, C.byref(rq), C.byref(rid)), "mh_server_submit")
        return rid.value

    def poll(self, rid: int):
        """Result dict, or None while the request is not finished."""
        res = Result()
        rc = _lib().mh_server_poll(self._h, rid, C.byref(res))
        if rc == ENOTREADY:
            return None
        _check(rc, "mh_server_poll")
        return {f: getattr(res, f) for f, _ in Result._fields_}

    def progress(self, rid: int) -> int:
        """Replicas finished so far (all of them once the request is done)."""
        res = Result()
        rc = _lib().mh_server_poll(self._h, rid, C.byref(res))
        if rc not in (0, ENOTREADY):
            _check(rc, "mh_server_poll")
        return res.replicas

    def close(self):
        if self._h:
            _lib().mh_server_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def time_kernels(assemblies, kind: int, launches: int = 50, reps: int = 20) -> float:
    """mh_time_kernels: mean microseconds of one step's launches of one kernel kind,
    replayed back to back on the plan of the assemblies' last run (kind 0 field sums,
    2 matrix product, 3 update, 4 matrix-form update; 3 and 4 overwrite the run's state)."""
    k = len(assemblies)
    hs = (C.c_void_p * k)(*[a._h.value for a in assemblies])
    us = C.c_double()
    _check(_lib().mh_time_kernels(hs, k, kind, launches, reps, C.byref(us)), "mh_time_kernels")
    return us.value


def run_batch(assemblies, n_replicas, seeds, stream=None):
    """mh_run_batch over several assemblies in one fused launch sequence."""
    k = len(assemblies)
    hs = (C.c_void_p * k)(*[a._h.value for a in assemblies])
    R = (C.c_int64 * k)(*n_replicas)
    S = (C.c_uint64 * k)(*seeds)
    _check(_lib().mh_run_batch(hs, k, R, S, stream), "mh_run_batch")
    for a, r in zip(assemblies, n_replicas):
        a.R = r


def params_from_material(mat, precision: int = FP64) -> Params:
    """Params from a workloads.Material."""
    return Params.make(precision=precision, **mat.as_dict())
