"""ctypes binding of libddcal (the C ABI in ``include/ddcal.h``).

Argument marshalling only: torch tensors provide device memory and the HIP stream
(``torch.cuda.current_stream()`` on ROCm is a hipStream_t); every step of the calibration
path runs in the library's HIP kernels.  If the library is missing, importing this module
raises: there is no fallback.

Layouts (see ``include/ddcal.h``): visibility-like tensors are ``[8, T, F, B]`` planes
(xx.re, xx.im, xy.re, xy.im, yx.re, yx.im, yy.re, yy.im), coherencies of K clusters are
``[K, 8, T, F, B]``, Jones are float64 ``[K, N, 8]``.
"""
from __future__ import annotations

import ctypes as ct
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libddcal.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with python -m paper_1910_13908_amd.build_lib")
_lib = ct.CDLL(LIB_PATH)

FP64 = 0
MIXED = 1

OK, EINVAL, ENOMEM, EDEVICE, ENOTPD, ENONFINITE, ETIMEOUT = 0, -1, -2, -3, -4, -5, -6
(TIMER_CHOLESKY, TIMER_PREDICT, TIMER_BUILD, TIMER_TRSV, TIMER_TRIAL, TIMER_MODEL, TIMER_REFINE,
 TIMER_ADJOINT, TIMER_PREDICT_FACTORED) = range(9)

EXPORTS = ("ddc_default_lm_opts", "ddc_create", "ddc_destroy", "ddc_set_stream", "ddc_last_error",
           "ddc_workspace_bytes", "ddc_predict", "ddc_predict_factored", "ddc_residual",
           "ddc_residual_noalloc", "ddc_add_model",
           "ddc_build_normal_eq", "ddc_damped_solve", "ddc_lm_solve", "ddc_calibrate",
           "ddc_cost_gradient", "ddc_set_wait_limit", "ddc_enable_timing", "ddc_enable_timers", "ddc_get_timing", "ddc_calibrate_footprint",
           "ddc_server_create", "ddc_server_destroy", "ddc_server_submit", "ddc_server_wait",
           "ddc_server_stats", "ddc_server_last_error")


class Obs(ct.Structure):
    _fields_ = [("n_stations", ct.c_int32), ("n_times", ct.c_int32), ("n_chans", ct.c_int32),
                ("u", ct.c_void_p), ("v", ct.c_void_p), ("w", ct.c_void_p), ("freq_hz", ct.c_void_p)]


class Sky(ct.Structure):
    _fields_ = [("n_clusters", ct.c_int32), ("cluster_offset", ct.POINTER(ct.c_int32)),
                ("l", ct.c_void_p), ("m", ct.c_void_p), ("I", ct.c_void_p), ("Q", ct.c_void_p),
                ("U", ct.c_void_p), ("V", ct.c_void_p)]


class LMOpts(ct.Structure):
    _fields_ = [("n_iter", ct.c_int32), ("precision", ct.c_int32), ("tau", ct.c_double),
                ("mu_floor", ct.c_double), ("refine_tol", ct.c_double), ("refine_max", ct.c_int32)]


class LMState(ct.Structure):
    _fields_ = [("mu", ct.c_double), ("nu", ct.c_double), ("fresh", ct.c_int32)]


class LMInfo(ct.Structure):
    _fields_ = [("cost0", ct.c_double), ("cost", ct.c_double), ("n_accept", ct.c_int32),
                ("n_reject", ct.c_int32), ("n_notpd", ct.c_int32), ("max_refine", ct.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class LMStep(ct.Structure):
    _fields_ = [("cost", ct.c_double), ("mu_eff", ct.c_double), ("mu", ct.c_double),
                ("nu", ct.c_double), ("accepted", ct.c_int32), ("refine_steps", ct.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class CalOpts(ct.Structure):
    _fields_ = [("n_sweeps", ct.c_int32), ("lm", LMOpts)]


_vp = ct.c_void_p
_lib.ddc_default_lm_opts.argtypes = [ct.POINTER(LMOpts)]
_lib.ddc_default_lm_opts.restype = None
_lib.ddc_create.argtypes = [ct.POINTER(_vp), ct.c_int32]
_lib.ddc_destroy.argtypes = [_vp]
_lib.ddc_set_stream.argtypes = [_vp, _vp]
_lib.ddc_last_error.argtypes = [_vp]
_lib.ddc_last_error.restype = ct.c_char_p
_lib.ddc_workspace_bytes.argtypes = [_vp]
_lib.ddc_workspace_bytes.restype = ct.c_int64
_lib.ddc_predict.argtypes = [_vp, ct.POINTER(Obs), ct.POINTER(Sky), ct.c_int32, _vp]
_lib.ddc_predict_factored.argtypes = [_vp, ct.POINTER(Obs), _vp, _vp, _vp, ct.POINTER(Sky),
                                      ct.c_int32, _vp]
_lib.ddc_residual.argtypes = [_vp, ct.POINTER(Obs), ct.c_int32, _vp, _vp, _vp, ct.c_int32, _vp,
                              ct.POINTER(ct.c_double)]
_lib.ddc_residual_noalloc.argtypes = [_vp, ct.POINTER(Obs), ct.c_int32, _vp, _vp, _vp, ct.c_int32,
                                      _vp, ct.POINTER(ct.c_double)]
_lib.ddc_add_model.argtypes = [_vp, ct.POINTER(Obs), ct.c_int32, _vp, _vp, _vp, ct.c_double,
                               ct.c_int32, _vp]
_lib.ddc_build_normal_eq.argtypes = [_vp, ct.POINTER(Obs), _vp, _vp, _vp, ct.c_int32, _vp, _vp,
                                     ct.POINTER(ct.c_double)]
_lib.ddc_damped_solve.argtypes = [_vp, ct.c_int32, _vp, _vp, ct.c_double, ct.c_int32, ct.c_double,
                                  ct.c_int32, _vp, ct.POINTER(ct.c_int32)]
_lib.ddc_lm_solve.argtypes = [_vp, ct.POINTER(Obs), _vp, _vp, _vp, ct.POINTER(LMOpts),
                              ct.POINTER(LMState), ct.POINTER(LMInfo), ct.POINTER(LMStep)]
_lib.ddc_calibrate.argtypes = [_vp, ct.POINTER(Obs), ct.POINTER(Sky), _vp, _vp, ct.POINTER(CalOpts),
                               _vp, ct.POINTER(LMInfo), ct.POINTER(LMStep)]
_lib.ddc_cost_gradient.argtypes = [_vp, ct.POINTER(Obs), ct.c_int32, _vp, _vp, _vp, ct.c_int32, _vp,
                                   ct.POINTER(ct.c_double)]
_lib.ddc_set_wait_limit.argtypes = [_vp, ct.c_uint32]
_lib.ddc_enable_timing.argtypes = [_vp, ct.c_int32]
_lib.ddc_enable_timers.argtypes = [_vp, ct.c_uint32]
_lib.ddc_get_timing.argtypes = [_vp, ct.c_int32, ct.POINTER(ct.c_int64), ct.POINTER(ct.c_double),
                                ct.POINTER(ct.c_double)]
_lib.ddc_calibrate_footprint.argtypes = [ct.POINTER(Obs), ct.c_int32, ct.c_int32, ct.c_int32,
                                         ct.c_int32]
_lib.ddc_calibrate_footprint.restype = ct.c_int64
_lib.ddc_server_create.argtypes = [ct.POINTER(_vp), ct.c_int32, ct.c_int32, ct.c_int64]
_lib.ddc_server_destroy.argtypes = [_vp]
_lib.ddc_server_submit.argtypes = [_vp, ct.POINTER(Obs), ct.POINTER(Sky), _vp, _vp, ct.POINTER(CalOpts),
                                   ct.POINTER(ct.c_int64)]
_lib.ddc_server_wait.argtypes = [_vp, ct.c_int64, ct.POINTER(LMInfo), ct.POINTER(ct.c_double),
                                 ct.POINTER(ct.c_double)]
_lib.ddc_server_stats.argtypes = [_vp, ct.POINTER(ct.c_int64), ct.POINTER(ct.c_int32), ct.POINTER(ct.c_int64)]
_lib.ddc_server_last_error.argtypes = [_vp]
_lib.ddc_server_last_error.restype = ct.c_char_p
for _f in EXPORTS:
    if _f not in ("ddc_default_lm_opts", "ddc_last_error", "ddc_workspace_bytes",
                  "ddc_calibrate_footprint", "ddc_server_last_error"):
        getattr(_lib, _f).restype = ct.c_int


class DdcError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"ddcal status {status}: {msg}")
        self.status = status


def default_lm_opts(**kw) -> LMOpts:
    o = LMOpts()
    _lib.ddc_default_lm_opts(ct.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr()


class Context:
    """A library context on one device; calls enqueue on torch's current stream."""

    def __init__(self, device: int = 0):
        import torch
        self._torch = torch
        h = _vp()
        st = _lib.ddc_create(ct.byref(h), device)
        if st != OK:
            raise DdcError(st, "ddc_create failed")
        self.h = h
        self.device = device

    def close(self):
        if getattr(self, "h", None):
            _lib.ddc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _bind(self):
        s = self._torch.cuda.current_stream(self.device).cuda_stream
        _lib.ddc_set_stream(self.h, _vp(s))

    def _check(self, st):
        if st != OK:
            raise DdcError(st, _lib.ddc_last_error(self.h).decode())

    def workspace_bytes(self) -> int:
        return int(_lib.ddc_workspace_bytes(self.h))

    # -- calls ---------------------------------------------------------------------------
    def predict(self, obs: "DeviceObs", sky: "DeviceSky", precision: int, out=None):
        torch = self._torch
        dt = torch.float32 if precision == MIXED else torch.float64
        if out is None:
            out = torch.empty((sky.K, 8, obs.T, obs.F, obs.B), dtype=dt, device=obs.u.device)
        self._bind()
        self._check(_lib.ddc_predict(self.h, ct.byref(obs.c), ct.byref(sky.c), precision, _ptr(out)))
        return out

    def predict_factored(self, obs: "DeviceObs", su, sv, sw, sky: "DeviceSky", precision: int,
                         out=None):
        """ddc_predict_factored: su, sv, sw are [T, N] float64 station coordinates (metres)."""
        torch = self._torch
        dt = torch.float32 if precision == MIXED else torch.float64
        for a in (su, sv, sw):
            if a.dtype != torch.float64 or not a.is_contiguous() or tuple(a.shape) != (obs.T, obs.N):
                raise ValueError("station coordinates must be contiguous float64 [T, N]")
        if out is None:
            out = torch.empty((sky.K, 8, obs.T, obs.F, obs.B), dtype=dt, device=obs.u.device)
        self._bind()
        self._check(_lib.ddc_predict_factored(self.h, ct.byref(obs.c), _ptr(su), _ptr(sv), _ptr(sw),
                                              ct.byref(sky.c), precision, _ptr(out)))
        return out

    def residual(self, obs, K, vis, coh, jones, precision, res=None, want_cost=True):
        self._bind()
        cost = ct.c_double(0.0)
        self._check(_lib.ddc_residual(self.h, ct.byref(obs.c), K, _ptr(vis), _ptr(coh), _ptr(jones),
                                      precision, _ptr(res), ct.byref(cost) if want_cost else None))
        return cost.value if want_cost else None

    def residual_noalloc(self, obs, K, vis, coh, jones, precision, res=None, want_cost=True):
        """ddc_residual_noalloc: ddc_residual with fixed device scratch (no allocation)."""
        self._bind()
        cost = ct.c_double(0.0)
        self._check(_lib.ddc_residual_noalloc(self.h, ct.byref(obs.c), K, _ptr(vis), _ptr(coh),
                                              _ptr(jones), precision, _ptr(res),
                                              ct.byref(cost) if want_cost else None))
        return cost.value if want_cost else None

    def add_model(self, obs, K, inp, coh, jones, alpha, precision, out):
        self._bind()
        self._check(_lib.ddc_add_model(self.h, ct.byref(obs.c), K, _ptr(inp), _ptr(coh), _ptr(jones),
                                       float(alpha), precision, _ptr(out)))
        return out

    def build_normal_eq(self, obs, y, coh_k, jones_k, precision, JtJ=None, Jtr=None):
        torch = self._torch
        n = 8 * obs.N
        dt = torch.float32 if precision == MIXED else torch.float64
        if JtJ is None:
            JtJ = torch.empty((n, n), dtype=dt, device=y.device)
        if Jtr is None:
            Jtr = torch.empty((n,), dtype=dt, device=y.device)
        cost = ct.c_double(0.0)
        self._bind()
        self._check(_lib.ddc_build_normal_eq(self.h, ct.byref(obs.c), _ptr(y), _ptr(coh_k), _ptr(jones_k),
                                             precision, _ptr(JtJ), _ptr(Jtr), ct.byref(cost)))
        return JtJ, Jtr, cost.value

    def damped_solve(self, H, g, mu, precision, refine_tol=1e-10, refine_max=5):
        torch = self._torch
        n = int(g.shape[0])
        d = torch.empty((n,), dtype=torch.float64, device=g.device)
        steps = ct.c_int32(0)
        self._bind()
        self._check(_lib.ddc_damped_solve(self.h, n, _ptr(H), _ptr(g), float(mu), precision,
                                          float(refine_tol), int(refine_max), _ptr(d), ct.byref(steps)))
        return d, steps.value

    def lm_solve(self, obs, y, coh_k, jones_k, opts: LMOpts, state: Optional[LMState] = None,
                 want_info=True, want_trace=False):
        """ddc_lm_solve; returns the LMInfo (or None), and with want_trace also the list of
        per-iteration LMStep records."""
        info = LMInfo()
        trace = (LMStep * max(1, opts.n_iter))() if want_trace else None
        self._bind()
        self._check(_lib.ddc_lm_solve(self.h, ct.byref(obs.c), _ptr(y), _ptr(coh_k), _ptr(jones_k),
                                      ct.byref(opts), ct.byref(state) if state is not None else None,
                                      ct.byref(info) if want_info else None, trace))
        out = info if want_info else None
        if want_trace:
            return out, list(trace)[:opts.n_iter]
        return out

    def calibrate(self, obs, sky, vis, jones, n_sweeps, lm: LMOpts, res=None, want_info=True,
                  want_trace=False):
        """ddc_calibrate; returns infos[sweep][cluster] (or None), and with want_trace also
        trace[sweep][cluster] = list of per-iteration LMStep records."""
        opts = CalOpts(n_sweeps=n_sweeps, lm=lm)
        infos = (LMInfo * max(1, n_sweeps * sky.K))()
        nit = lm.n_iter
        trace = (LMStep * max(1, n_sweeps * sky.K * nit))() if want_trace else None
        self._bind()
        self._check(_lib.ddc_calibrate(self.h, ct.byref(obs.c), ct.byref(sky.c), _ptr(vis), _ptr(jones),
                                       ct.byref(opts), _ptr(res), infos if want_info else None,
                                       trace))
        out = None
        if want_info:
            out = [[infos[e * sky.K + k] for k in range(sky.K)] for e in range(n_sweeps)]
        if want_trace:
            tr = [[list(trace[(e * sky.K + k) * nit:(e * sky.K + k + 1) * nit]) for k in range(sky.K)]
                  for e in range(n_sweeps)]
            return out, tr
        return out

    def cost_gradient(self, obs, K, vis, coh, jones, precision, grad=None, want_cost=True):
        """f and df/d(jones) ([K, N, 8] float64) from the adjoint kernel."""
        if grad is None:
            grad = self._torch.empty_like(jones)
        cost = ct.c_double(0.0)
        self._bind()
        self._check(_lib.ddc_cost_gradient(self.h, ct.byref(obs.c), K, _ptr(vis), _ptr(coh), _ptr(jones),
                                           precision, _ptr(grad), ct.byref(cost) if want_cost else None))
        return (cost.value if want_cost else None), grad

    def set_wait_limit(self, polls: int):
        """ddc_set_wait_limit: bound every inter-workgroup wait at `polls` polls (0: default)."""
        self._check(_lib.ddc_set_wait_limit(self.h, int(polls)))

    def enable_timing(self, on=True, timers=None):
        """Time every kernel class (on), none, or only those listed in timers (TIMER_*)."""
        if timers is None:
            self._check(_lib.ddc_enable_timing(self.h, 1 if on else 0))
        else:
            mask = 0
            for t in timers:
                mask |= 1 << t
            self._check(_lib.ddc_enable_timers(self.h, mask if on else 0))

    def timing(self, which):
        n = ct.c_int64(0)
        ms = ct.c_double(0.0)
        work = ct.c_double(0.0)
        self._check(_lib.ddc_get_timing(self.h, which, ct.byref(n), ct.byref(ms), ct.byref(work)))
        return n.value, ms.value, work.value


def calibrate_footprint(obs: "DeviceObs", n_clusters: int, n_sweeps: int, n_iter: int,
                        precision: int) -> int:
    return int(_lib.ddc_calibrate_footprint(ct.byref(obs.c), n_clusters, n_sweeps, n_iter,
                                            precision))


class Server:
    """Continuous-batching calibration server (see ddc_server_* in include/ddcal.h).

    ``submit`` keeps references to the request's tensors until ``wait`` returns, so the
    device memory stays valid while the library uses it.
    """

    def __init__(self, device: int = 0, n_slots: int = 4, hbm_budget_bytes: int = 16 << 30):
        h = _vp()
        st = _lib.ddc_server_create(ct.byref(h), device, n_slots, int(hbm_budget_bytes))
        if st != OK:
            raise DdcError(st, "ddc_server_create failed")
        self.h = h
        self._keep = {}

    def close(self):
        if getattr(self, "h", None):
            _lib.ddc_server_destroy(self.h)
            self.h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, obs: "DeviceObs", sky: "DeviceSky", vis, jones, n_sweeps: int, lm: LMOpts) -> int:
        opts = CalOpts(n_sweeps=n_sweeps, lm=lm)
        rid = ct.c_int64(0)
        st = _lib.ddc_server_submit(self.h, ct.byref(obs.c), ct.byref(sky.c), _ptr(vis), _ptr(jones),
                                    ct.byref(opts), ct.byref(rid))
        if st != OK:
            raise DdcError(st, _lib.ddc_server_last_error(self.h).decode())
        self._keep[rid.value] = (obs, sky, vis, jones, n_sweeps * sky.K)
        return rid.value

    def wait(self, rid: int):
        obs, sky, vis, jones, n_info = self._keep[rid]
        infos = (LMInfo * max(1, n_info))()
        lat = ct.c_double(0.0)
        que = ct.c_double(0.0)
        st = _lib.ddc_server_wait(self.h, rid, infos, ct.byref(lat), ct.byref(que))
        del self._keep[rid]
        if st != OK:
            raise DdcError(st, _lib.ddc_server_last_error(self.h).decode())
        return list(infos)[:n_info], lat.value, que.value

    def stats(self):
        n = ct.c_int64(0)
        m = ct.c_int32(0)
        p = ct.c_int64(0)
        _lib.ddc_server_stats(self.h, ct.byref(n), ct.byref(m), ct.byref(p))
        return {"completed": n.value, "max_running": m.value, "peak_arena_bytes": p.value}


# -- marshalling helpers ------------------------------------------------------------------

class DeviceObs:
    """Observation geometry as device tensors plus the ddc_obs struct pointing at them."""

    def __init__(self, u, v, w, freqs, n_stations: int):
        self.u, self.v, self.w, self.freqs = u, v, w, freqs
        self.N = int(n_stations)
        self.T = int(u.shape[0])
        self.B = int(u.shape[1])
        self.F = int(freqs.shape[0])
        if self.B != self.N * (self.N - 1) // 2:
            raise ValueError("u must be [T, N(N-1)/2]")
        self.c = Obs(self.N, self.T, self.F, _ptr(u), _ptr(v), _ptr(w), _ptr(freqs))


class DeviceSky:
    def __init__(self, l, m, I, Q, U, V, cluster_offset: Sequence[int]):
        self.l, self.m, self.I, self.Q, self.U, self.V = l, m, I, Q, U, V
        self.offs = (ct.c_int32 * len(cluster_offset))(*[int(x) for x in cluster_offset])
        self.K = len(cluster_offset) - 1
        self.c = Sky(self.K, self.offs, _ptr(l), _ptr(m), _ptr(I), _ptr(Q), _ptr(U), _ptr(V))


def device_obs(ob, device="cuda"):
    """DeviceObs from a synth.Obs (uvw and frequencies copied to the device)."""
    import torch
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=device)
    return DeviceObs(t(ob.u), t(ob.v), t(ob.w), t(ob.freqs), ob.N)


def device_station_uvw(ob, device="cuda"):
    """(su, sv, sw): station coordinates [T, N] float64 on the device, from a synth.Obs."""
    import torch
    return tuple(torch.as_tensor(np.ascontiguousarray(ob.suvw[..., i]), dtype=torch.float64,
                                 device=device) for i in range(3))


def device_sky(ob, device="cuda"):
    import torch
    t = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=device)
    return DeviceSky(t(ob.l), t(ob.m), t(ob.I), t(ob.Q), t(ob.U), t(ob.V), list(ob.cluster_offset))


def planes(x):
    """complex [..., T, F, B, 2, 2] -> real [..., 8, T, F, B] (NumPy)."""
    x = np.asarray(x)
    lead = x.shape[:-5]
    T, F, B = x.shape[-5:-2]
    flat = x.reshape(lead + (T, F, B, 4))
    out = np.empty(lead + (8, T, F, B))
    for e in range(4):
        out[..., 2 * e, :, :, :] = flat[..., e].real
        out[..., 2 * e + 1, :, :, :] = flat[..., e].imag
    return out


def unplanes(p):
    """real [..., 8, T, F, B] -> complex [..., T, F, B, 2, 2] (NumPy)."""
    p = np.asarray(p, dtype=np.float64)
    lead = p.shape[:-4]
    T, F, B = p.shape[-3:]
    out = np.empty(lead + (T, F, B, 4), dtype=np.complex128)
    for e in range(4):
        out[..., e] = p[..., 2 * e, :, :, :] + 1j * p[..., 2 * e + 1, :, :, :]
    return out.reshape(lead + (T, F, B, 2, 2))


def jones_real(J):
    """complex [..., N, 2, 2] -> float64 [..., N, 8] in (entry, re/im) order."""
    J = np.asarray(J)
    flat = J.reshape(J.shape[:-2] + (4,))
    out = np.empty(J.shape[:-2] + (8,))
    out[..., 0::2] = flat.real
    out[..., 1::2] = flat.imag
    return out


def jones_complex(x):
    x = np.asarray(x, dtype=np.float64)
    z = x[..., 0::2] + 1j * x[..., 1::2]
    return z.reshape(x.shape[:-1] + (2, 2))
