"""Thin ctypes binding of libesp.so with the C ABI's names.

Argument marshalling only: every step of the pipeline runs in the HIP
library. Device buffers are torch tensors on the plan's GPU; their data
pointers are handed to the library. A plan given a torch stream
(Plan(..., stream=s)) enqueues on it, and calls made while that stream is
torch's current stream need no ordering; otherwise the plan's stream is
ordered after torch's current stream before each call (and torch's stream
after it).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libesp.so")
_lib = None

STATUS = {0: "ESP_OK", -1: "ESP_E_INVALID", -2: "ESP_E_UNSUPPORTED", -3: "ESP_E_NOT_NEUTRAL",
          -4: "ESP_E_NOMEM", -5: "ESP_E_DEVICE", -6: "ESP_E_BUSY"}


class EspError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class esp_params(C.Structure):
    _fields_ = [("nf", C.c_int), ("P", C.c_int), ("degree", C.c_int), ("precision", C.c_int),
                ("tile", C.c_int), ("fft_passes", C.c_int),
                ("c", C.c_double), ("c1", C.c_double), ("rc", C.c_double), ("h_max", C.c_double),
                ("kappa", C.c_double), ("L", C.c_double), ("h", C.c_double), ("tol", C.c_double),
                ("s0", C.c_double), ("force_method", C.c_int), ("local", C.c_int),
                ("method", C.c_int), ("Ly", C.c_double), ("Lz", C.c_double),
                ("xy", C.c_double), ("xz", C.c_double), ("yz", C.c_double),
                ("stream", C.c_void_p), ("deterministic", C.c_int)]

    def to_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class esp_server_opts(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_size_t), ("max_active", C.c_int), ("keep_outputs", C.c_int)]


class esp_request(C.Structure):
    _fields_ = [("L", C.c_double), ("N", C.c_int64), ("tol", C.c_double), ("pos", C.c_void_p),
                ("q", C.c_void_p), ("nsteps", C.c_int), ("drift", C.c_double), ("seed", C.c_uint64),
                ("tag", C.c_uint64)]


class esp_result(C.Structure):
    _fields_ = [("id", C.c_uint64), ("tag", C.c_uint64), ("status", C.c_int), ("nsteps", C.c_int),
                ("N", C.c_int64), ("nf", C.c_int), ("P", C.c_int), ("t_submit", C.c_double),
                ("t_admit", C.c_double), ("t_done", C.c_double), ("E_first", C.c_double), ("E_last", C.c_double)]

    def to_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class esp_server_stats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("admitted", C.c_int64), ("completed", C.c_int64),
                ("failed", C.c_int64), ("active", C.c_int64), ("waiting", C.c_int64), ("iterations", C.c_int64),
                ("particle_steps", C.c_double), ("busy_s", C.c_double), ("span_s", C.c_double),
                ("p50_latency_s", C.c_double), ("p99_latency_s", C.c_double), ("max_latency_s", C.c_double),
                ("bytes_in_use", C.c_size_t), ("bytes_peak", C.c_size_t), ("build_s", C.c_double),
                ("admit_s", C.c_double), ("step_s", C.c_double)]

    def to_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_P = C.POINTER
_vp = C.c_void_p
_SIGS = {
    "esp_plan_query": (C.c_int, [_P(C.c_double), C.c_int64, C.c_double, _P(esp_params), _P(esp_params)]),
    "esp_window_coeffs": (C.c_int, [_P(esp_params), _P(C.c_double)]),
    "esp_influence_tables": (C.c_int, [_P(esp_params), _P(C.c_double), _P(C.c_double)]),
    "esp_local_kernel": (C.c_int, [_P(esp_params), _P(C.c_double), C.c_int64, _P(C.c_double), _P(C.c_double)]),
    "esp_warm_tables": (C.c_int, [_P(C.c_double), C.c_int, C.c_int, C.c_int]),
    "esp_local_coeffs": (C.c_int, [_P(esp_params), _P(C.c_double), _P(C.c_double), _P(C.c_int), _P(C.c_int)]),
    "esp_num_phases": (C.c_int, []),
    "esp_plan_create": (C.c_int, [_P(C.c_double), C.c_int64, C.c_double, _P(_vp)]),
    "esp_plan_create_ex": (C.c_int, [_P(C.c_double), C.c_int64, C.c_double, _P(esp_params), _P(_vp)]),
    "esp_batch_create": (C.c_int, [C.c_int, _P(C.c_double), _P(C.c_int64), _P(C.c_double), _P(esp_params),
                                   _P(_vp)]),
    "esp_plan_get_params": (C.c_int, [_vp, C.c_int, _P(esp_params)]),
    "esp_plan_num_systems": (C.c_int, [_vp]),
    "esp_plan_stream": (_vp, [_vp]),
    "esp_plan_set_stream": (C.c_int, [_vp, _vp]),
    "esp_plan_shortrange_coeffs": (C.c_int, [_vp, _P(C.c_double), _P(C.c_int), _P(C.c_int)]),
    "esp_batch_longrange": (C.c_int, [_vp, _vp, _vp, _vp, _vp, _P(C.c_double)]),
    "esp_longrange": (C.c_int, [_vp, _vp, _vp, _vp, _vp, _P(C.c_double)]),
    "esp_longrange_async": (C.c_int, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "esp_plan_sync": (C.c_int, [_vp]),
    "esp_longrange_noalloc": (C.c_int, [_P(C.c_double), C.c_int64, C.c_double, _P(esp_params), _vp, _vp, _vp, _vp,
                                        _P(C.c_double), _vp]),
    "esp_plan_set_graph": (C.c_int, [_vp, C.c_int]),
    "esp_plan_autotune": (C.c_int, [_vp, _vp, _vp, _vp, _vp, C.c_int, _P(C.c_int)]),
    "esp_plan_destroy": (None, [_vp]),
    "esp_debug_stage": (C.c_int, [_vp, _vp, _vp, _vp, C.c_int, _vp]),
    "esp_debug_gather": (C.c_int, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "esp_plan_profile": (C.c_int, [_vp, _vp, _vp, _vp, _vp, C.c_int, _P(C.c_double)]),
    "esp_phase_name": (C.c_char_p, [C.c_int]),
    "esp_plan_profile_launches": (C.c_int, [_vp, _vp, _vp, _vp, _vp, C.c_int, C.c_int, C.c_int, _P(C.c_double),
                                            _P(C.c_int64), _P(C.c_int64), _P(C.c_int64), _P(C.c_int)]),
    "esp_server_create": (C.c_int, [_P(esp_server_opts), _P(_vp)]),
    "esp_server_submit": (C.c_int, [_vp, _P(esp_request), _P(C.c_uint64)]),
    "esp_server_poll": (C.c_int, [_vp, _P(esp_result), C.c_int, _P(C.c_int)]),
    "esp_server_fetch": (C.c_int, [_vp, C.c_uint64, _vp, _vp]),
    "esp_server_wait": (C.c_int, [_vp, C.c_double]),
    "esp_server_get_stats": (C.c_int, [_vp, _P(esp_server_stats)]),
    "esp_server_destroy": (None, [_vp]),
    "esp_server_last_error": (C.c_char_p, []),
    "esp_last_error": (C.c_char_p, []),
    "esp_version": (C.c_char_p, []),
}


def lib():
    """Load libesp.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"{_LIB_PATH} is missing: build it with python -m paper_2505_09727_amd.build")
        L = C.CDLL(_LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(status):
    if status != 0:
        raise EspError(status, lib().esp_last_error().decode())


def _stream_handle(stream):
    """hipStream_t of a torch stream (or a raw handle)."""
    return stream if isinstance(stream, int) else stream.cuda_stream


def _req(**kw) -> esp_params:
    p = esp_params()
    for k, v in kw.items():
        if v is not None:
            setattr(p, k, _stream_handle(v) if k == "stream" else v)
    return p


def _box(L):
    return (C.c_double * 3)(L, L, L)


def esp_version() -> str:
    return lib().esp_version().decode()


def esp_plan_query(box, N, tol, **req):
    """Resolved parameters (dict) for a cubic box; host only."""
    b = (C.c_double * 3)(*box) if np.ndim(box) else _box(float(box))
    out = esp_params()
    _check(lib().esp_plan_query(b, int(N), float(tol), C.byref(_req(**req)), C.byref(out)))
    return out


def esp_window_coeffs(params: esp_params) -> np.ndarray:
    c = np.zeros(params.P * (params.degree + 1))
    _check(lib().esp_window_coeffs(C.byref(params), c.ctypes.data_as(_P(C.c_double))))
    return c.reshape(params.P, params.degree + 1)


def esp_influence_tables(params: esp_params):
    h2 = params.nf // 2
    TS = np.zeros(3 * h2 * h2 + 1)
    Tphi = np.zeros(h2 + 1)
    _check(lib().esp_influence_tables(C.byref(params), TS.ctypes.data_as(_P(C.c_double)),
                                      Tphi.ctypes.data_as(_P(C.c_double))))
    return TS, Tphi


def esp_local_kernel(params: esp_params, r):
    r = np.ascontiguousarray(r, dtype=np.float64)
    Lr, dLr = np.zeros_like(r), np.zeros_like(r)
    dp = _P(C.c_double)
    _check(lib().esp_local_kernel(C.byref(params), r.ctypes.data_as(dp), len(r), Lr.ctypes.data_as(dp),
                                  dLr.ctypes.data_as(dp)))
    return Lr, dLr


ESP_LOCAL_COEF_MAX = 104


def esp_local_coeffs(params: esp_params):
    """Piecewise polynomials (A, B), each pieces x (degree + 1), that the
    device evaluates for the local part in grid units (esp.h)."""
    A = np.zeros(ESP_LOCAL_COEF_MAX)
    B = np.zeros(ESP_LOCAL_COEF_MAX)
    K, d = C.c_int(0), C.c_int(0)
    dp = _P(C.c_double)
    _check(lib().esp_local_coeffs(C.byref(params), A.ctypes.data_as(dp), B.ctypes.data_as(dp), C.byref(K),
                                  C.byref(d)))
    m = K.value * (d.value + 1)
    return A[:m].reshape(K.value, d.value + 1), B[:m].reshape(K.value, d.value + 1)


def esp_warm_tables(tols, nf_max: int = 144, threads: int = 0) -> None:
    """Precompute the parameter classes of every grid size up to nf_max for
    each tolerance (host threads; process-wide cache)."""
    arr = (C.c_double * len(tols))(*[float(t) for t in tols])
    _check(lib().esp_warm_tables(arr, len(tols), int(nf_max), int(threads)))


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def esp_longrange_noalloc(box, pos, q, phi=None, F=None, tol=1e-4, stream=None, **req):
    """One evaluation with no device allocation (esp_longrange_noalloc) on
    torch tensors; runs on `stream` (a torch stream, default torch's current
    one) and returns the energy."""
    import torch
    st = torch.cuda.current_stream() if stream is None else stream
    b = (C.c_double * 3)(*box) if np.ndim(box) else _box(float(box))
    E = C.c_double(0.0)
    _check(lib().esp_longrange_noalloc(b, int(q.shape[0]), float(tol), C.byref(_req(**req)), _ptr(pos), _ptr(q),
                                       _ptr(phi), _ptr(F), C.byref(E), C.c_void_p(_stream_handle(st))))
    return E.value


class Plan:
    """A single-system or batched plan (esp_plan_create_ex / esp_batch_create)."""

    def __init__(self, L, N, tol, per_system=None, **req):
        """Single system (scalar L, a box (Lx, Ly, Lz) or a triclinic cell
        (Lx, Ly, Lz, xy, xz, yz), and scalar N) or batch (sequences of x sides
        and sizes; per-system Ly, Lz and tilts through per_system).
        per_system: one dict of requested parameters per system of a batch
        (overrides req)."""
        self._h = C.c_void_p()
        if np.ndim(L) == 0 or (np.ndim(N) == 0 and len(L) in (3, 6)):
            # one system: side L, an orthorhombic box or a triclinic cell
            if np.ndim(L) and len(L) == 6:
                req = dict(req, xy=float(L[3]), xz=float(L[4]), yz=float(L[5]))
                L = L[:3]
            box = _box(float(L)) if np.ndim(L) == 0 else (C.c_double * 3)(*[float(x) for x in L])
            _check(lib().esp_plan_create_ex(box, int(N), float(tol), C.byref(_req(**req)), C.byref(self._h)))
        else:
            Ls = np.ascontiguousarray(L, dtype=np.float64)
            Ns = np.ascontiguousarray(N, dtype=np.int64)
            tols = np.ascontiguousarray(np.broadcast_to(tol, Ls.shape), dtype=np.float64)
            kws = per_system if per_system is not None else [req] * len(Ls)
            reqs = (esp_params * len(Ls))(*[_req(**kw) for kw in kws])
            _check(lib().esp_batch_create(len(Ls), Ls.ctypes.data_as(_P(C.c_double)),
                                          Ns.ctypes.data_as(_P(C.c_int64)), tols.ctypes.data_as(_P(C.c_double)),
                                          reqs, C.byref(self._h)))
        self.nsys = lib().esp_plan_num_systems(self._h)
        self.params = [self.get_params(s) for s in range(self.nsys)]
        self.precision = self.params[0].precision

    def get_params(self, sys: int = 0) -> esp_params:
        out = esp_params()
        _check(lib().esp_plan_get_params(self._h, sys, C.byref(out)))
        return out

    @property
    def stream(self):
        return lib().esp_plan_stream(self._h)

    def set_stream(self, stream):
        """esp_plan_set_stream: enqueue later work on a torch stream (or handle)."""
        _check(lib().esp_plan_set_stream(self._h, C.c_void_p(_stream_handle(stream))))
        self.params = [self.get_params(s) for s in range(self.nsys)]

    def _order_after_torch(self):
        """Order the plan's stream after torch's current one; None when they
        are the same stream (nothing to order)."""
        import torch
        cur = torch.cuda.current_stream()
        if (self.stream or 0) == cur.cuda_stream:
            return None
        ext = torch.cuda.ExternalStream(self.stream)
        ext.wait_stream(cur)
        return ext

    @staticmethod
    def _order_torch_after(ext):
        if ext is not None:
            import torch
            torch.cuda.current_stream().wait_stream(ext)

    def longrange(self, pos, q, phi=None, F=None, energy=True):
        """Enqueue esp_longrange; returns the energies (numpy, one per system) or None."""
        ext = self._order_after_torch()
        E = (C.c_double * self.nsys)() if energy else None
        st = lib().esp_longrange(self._h, _ptr(pos), _ptr(q), _ptr(phi), _ptr(F), E)
        self._order_torch_after(ext)
        _check(st)
        return np.array(E[:]) if energy else None

    def batch_longrange(self, pos, q, phi=None, F=None, energy=True):
        """esp_batch_longrange: all systems of a batch plan (concatenated
        arrays); returns the per-system energies (numpy) or None."""
        ext = self._order_after_torch()
        E = (C.c_double * self.nsys)() if energy else None
        st = lib().esp_batch_longrange(self._h, _ptr(pos), _ptr(q), _ptr(phi), _ptr(F), E)
        self._order_torch_after(ext)
        _check(st)
        return np.array(E[:]) if energy else None

    def longrange_async(self, pos, q, phi=None, F=None, E_dev=None):
        ext = self._order_after_torch()
        st = lib().esp_longrange_async(self._h, _ptr(pos), _ptr(q), _ptr(phi), _ptr(F), _ptr(E_dev))
        self._order_torch_after(ext)
        _check(st)

    def shortrange_coeffs(self):
        """esp_plan_shortrange_coeffs: the (A, B) piecewise polynomials of the
        local kernel L(r), L'(r) of system 0, in grid units (esp.h)."""
        coef = np.zeros(2 * ESP_LOCAL_COEF_MAX)
        K, d = C.c_int(0), C.c_int(0)
        _check(lib().esp_plan_shortrange_coeffs(self._h, coef.ctypes.data_as(_P(C.c_double)), C.byref(K),
                                                C.byref(d)))
        m = K.value * (d.value + 1)
        return coef[:m].reshape(K.value, d.value + 1), coef[m:2 * m].reshape(K.value, d.value + 1)

    def sync(self):
        _check(lib().esp_plan_sync(self._h))

    def set_graph(self, enable: bool = True):
        _check(lib().esp_plan_set_graph(self._h, int(bool(enable))))

    def autotune(self, pos, q, phi=None, F=None, reps: int = 3):
        """esp_plan_autotune: time the admissible bin edges per (grid, P) group
        on these buffers and rebuild the plan with the fastest; returns the
        chosen bin edge of every system."""
        ext = self._order_after_torch()
        tiles = (C.c_int * self.nsys)()
        st = lib().esp_plan_autotune(self._h, _ptr(pos), _ptr(q), _ptr(phi), _ptr(F), int(reps), tiles)
        self._order_torch_after(ext)
        _check(st)
        self.params = [self.get_params(s) for s in range(self.nsys)]
        return list(tiles)

    def debug_stage(self, pos, q, stage, out, grid_in=None):
        ext = self._order_after_torch()
        st = lib().esp_debug_stage(self._h, _ptr(pos), _ptr(q), _ptr(grid_in), int(stage), _ptr(out))
        self._order_torch_after(ext)
        _check(st)

    def debug_gather(self, pos, q, grid_c, phi=None, F=None):
        """esp_debug_gather: interpolate the caller's potential grid alone."""
        ext = self._order_after_torch()
        st = lib().esp_debug_gather(self._h, _ptr(pos), _ptr(q), _ptr(grid_c), _ptr(phi), _ptr(F))
        self._order_torch_after(ext)
        _check(st)

    def profile_launches(self, pos, q, phi, F, reps: int, phase: str):
        """esp_plan_profile_launches: mean ms, particles, grid points and
        workgroups of each launch of the "spread" or "gather" phase."""
        names = [lib().esp_phase_name(i).decode() for i in range(lib().esp_num_phases())]
        mx = 64
        ms, cnt = (C.c_double * mx)(), C.c_int()
        pa, pt, bl = (C.c_int64 * mx)(), (C.c_int64 * mx)(), (C.c_int64 * mx)()
        ext = self._order_after_torch()
        st = lib().esp_plan_profile_launches(self._h, _ptr(pos), _ptr(q), _ptr(phi), _ptr(F), int(reps),
                                             names.index(phase), mx, ms, pa, pt, bl, C.byref(cnt))
        self._order_torch_after(ext)
        _check(st)
        return [dict(ms=ms[k], particles=pa[k], points=pt[k], blocks=bl[k]) for k in range(cnt.value)]

    def close(self):
        if self._h:
            lib().esp_plan_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _scheck(status):
    if status != 0:
        raise EspError(status, lib().esp_server_last_error().decode())


class Server:
    """Continuous-batching request server (esp_server_*); FP32, host inputs."""

    def __init__(self, hbm_budget_bytes=0, max_active=0, keep_outputs=False):
        self._h = C.c_void_p()
        o = esp_server_opts(hbm_budget_bytes, max_active, int(bool(keep_outputs)))
        _scheck(lib().esp_server_create(C.byref(o), C.byref(self._h)))

    def submit(self, pos, q, L, tol, nsteps=1, drift=0.0, seed=0, tag=0):
        pos = np.ascontiguousarray(pos, dtype=np.float32)
        q = np.ascontiguousarray(q, dtype=np.float32)
        r = esp_request(float(L), len(q), float(tol), pos.ctypes.data, q.ctypes.data, int(nsteps), float(drift),
                        int(seed), int(tag))
        rid = C.c_uint64()
        _scheck(lib().esp_server_submit(self._h, C.byref(r), C.byref(rid)))
        return rid.value

    def poll(self, max_results=1024):
        buf = (esp_result * max_results)()
        n = C.c_int()
        _scheck(lib().esp_server_poll(self._h, buf, max_results, C.byref(n)))
        return [buf[i].to_dict() for i in range(n.value)]

    def fetch(self, rid, N):
        phi = np.empty(N, dtype=np.float32)
        F = np.empty((N, 3), dtype=np.float32)
        _scheck(lib().esp_server_fetch(self._h, rid, phi.ctypes.data, F.ctypes.data))
        return phi, F

    def wait(self, timeout_s=60.0):
        _scheck(lib().esp_server_wait(self._h, float(timeout_s)))

    def stats(self):
        st = esp_server_stats()
        _scheck(lib().esp_server_get_stats(self._h, C.byref(st)))
        return st.to_dict()

    def close(self):
        if self._h:
            lib().esp_server_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
