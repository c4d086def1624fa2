"""ctypes binding of ``libfgl.so`` (declared in include/fgl.h).

Argument marshalling only: every step of the likelihood runs in the HIP
library.  If the library has not been built, importing this module raises:
there is no other implementation to fall back to.

Function names mirror the C-ABI (``fgl_model_create``, ``fgl_loglike_batch``,
``fgl_serve_submit`` ...); ``Model`` and ``Server`` wrap them for numpy arrays
(host) and torch tensors (device memory and streams).
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfgl.so")

FGL_OK, FGL_EINVAL, FGL_ENOMEM, FGL_EBUSY, FGL_EDEVICE, FGL_EAGAIN = 0, -1, -2, -3, -4, -5
FGL_ECANCELED, FGL_ETIMEDOUT = -6, -7
FGL_PREC_MIXED, FGL_PREC_FP32, FGL_PREC_FP64 = 0, 1, 2
FGL_NO_21CM = 1
FGL_MIXED_DIRECT = 2
FGL_PLAIN_PROJECTED = 4
FGL_FORM_DIRECT, FGL_FORM_PROJECTED, FGL_FORM_THIN = 0, 1, 2
PREC = {"mixed": FGL_PREC_MIXED, "fp32": FGL_PREC_FP32, "fp64": FGL_PREC_FP64}
_NAMES = {FGL_EINVAL: "EINVAL", FGL_ENOMEM: "ENOMEM", FGL_EBUSY: "EBUSY",
          FGL_EDEVICE: "EDEVICE", FGL_EAGAIN: "EAGAIN"}


class FGLError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with `python -m paper_2603_13196_amd.build` "
        "(the likelihood has no implementation outside the HIP library)")

# torch bundles its own HIP runtime under the same soname as ROCm's; loading
# torch first makes libfgl.so bind to that runtime, so the process has
# exactly one HIP runtime and torch tensors/streams can be handed over.
try:
    import torch  # noqa: F401
except ImportError:
    pass

_lib = ctypes.CDLL(LIB_PATH)
_dp = ctypes.POINTER(ctypes.c_double)
_fp = ctypes.POINTER(ctypes.c_float)
_vp = ctypes.c_void_p

_SIGS = {
    "fgl_model_create": ([_fp, _dp, _dp, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                          ctypes.c_int, ctypes.c_double, ctypes.c_uint,
                          ctypes.POINTER(_vp)], ctypes.c_int),
    "fgl_model_create_masks": ([_fp, _dp, _dp, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_uint,
                                ctypes.POINTER(_vp)], ctypes.c_int),
    "fgl_model_nparams": ([_vp], ctypes.c_int),
    "fgl_mixed_form": ([_vp], ctypes.c_int),
    "fgl_loglike_batch": ([_vp, _dp, ctypes.c_int, _dp, ctypes.c_int], ctypes.c_int),
    "fgl_loglike_batch_device": ([_vp, _vp, ctypes.c_int, _vp, ctypes.c_int, _vp],
                                 ctypes.c_int),
    "fgl_loglike_batch_device_noalloc": ([_vp, _vp, ctypes.c_int, _vp, ctypes.c_int, _vp],
                                         ctypes.c_int),
    "fgl_loglike_grad_batch": ([_vp, _dp, ctypes.c_int, _dp, _dp, ctypes.c_int], ctypes.c_int),
    "fgl_loglike_grad_batch_device": ([_vp, _vp, ctypes.c_int, _vp, _vp, ctypes.c_int, _vp],
                                      ctypes.c_int),
    "fgl_get_tile": ([_vp, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                      ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)],
                     ctypes.c_int),
    "fgl_tune": ([_vp, ctypes.c_int, ctypes.c_int], ctypes.c_int),
    "fgl_set_tile": ([_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                      ctypes.c_int], ctypes.c_int),
    "fgl_model_bytes": ([_vp], ctypes.c_size_t),
    "fgl_model_destroy": ([_vp], ctypes.c_int),
    "fgl_kernel_timing": ([_vp, ctypes.c_int], ctypes.c_int),
    "fgl_kernel_time": ([_vp, _dp, ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
    "fgl_serve_create": ([ctypes.c_size_t, ctypes.c_int, ctypes.POINTER(_vp)], ctypes.c_int),
    "fgl_serve_submit": ([_vp, _vp, _dp, ctypes.c_int, _dp, ctypes.c_int,
                          ctypes.POINTER(ctypes.c_uint64)], ctypes.c_int),
    "fgl_serve_poll": ([_vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int), _dp],
                       ctypes.c_int),
    "fgl_serve_drain": ([_vp], ctypes.c_int),
    "fgl_serve_hold": ([_vp, ctypes.c_int], ctypes.c_int),
    "fgl_serve_cancel": ([_vp, ctypes.c_uint64], ctypes.c_int),
    "fgl_serve_set_timeout": ([_vp, ctypes.c_double], ctypes.c_int),
    "fgl_serve_set_sharing": ([_vp, ctypes.c_int], ctypes.c_int),
    "fgl_serve_stats": ([_vp, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64),
                         ctypes.POINTER(ctypes.c_uint64)], ctypes.c_int),
    "fgl_serve_destroy": ([_vp], ctypes.c_int),
    "fgl_chains_create": ([_vp, ctypes.c_int, _dp, _dp, ctypes.c_uint64, ctypes.POINTER(_vp)],
                          ctypes.c_int),
    "fgl_chains_run": ([_vp, _dp, _dp, ctypes.c_int, ctypes.c_double, _dp, ctypes.c_int,
                        ctypes.c_int, _dp, _dp, ctypes.POINTER(ctypes.c_int64),
                        ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
    "fgl_chains_destroy": ([_vp], ctypes.c_int),
    "fgl_chains_philox": ([ctypes.POINTER(ctypes.c_uint32), ctypes.c_int, ctypes.c_uint32,
                           ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint32)], ctypes.c_int),
    "fgl_sky_create": ([ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp, _dp, _dp, _fp,
                        ctypes.POINTER(ctypes.c_uint8), _dp, ctypes.c_double, ctypes.c_double,
                        ctypes.POINTER(_vp)], ctypes.c_int),
    "fgl_sky_importance": ([_vp, ctypes.POINTER(ctypes.c_int32), ctypes.c_int, ctypes.c_int, _dp],
                           ctypes.c_int),
    "fgl_partition": ([_dp, _dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp], ctypes.c_int),
    "fgl_sky_chromatic": ([_vp, _dp, ctypes.c_int, ctypes.POINTER(ctypes.c_int32), ctypes.c_int,
                           _dp], ctypes.c_int),
    "fgl_sky_kernel_ms": ([_vp, _dp], ctypes.c_int),
    "fgl_sky_destroy": ([_vp], ctypes.c_int),
    "fgl_noise_loglike": ([ctypes.c_int64, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                           ctypes.c_uint64, _dp, _dp], ctypes.c_int),
    "fgl_noise_quantile": ([_dp, ctypes.c_int, _dp, ctypes.c_int, _dp], ctypes.c_int),
    "fgl_tune_cache": ([ctypes.c_char_p], ctypes.c_int),
    "fgl_last_error": ([], ctypes.c_char_p),
}
for _name, (_args, _res) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _res

EXPORTED = tuple(_SIGS)


def _check(rc: int) -> int:
    if rc != FGL_OK:
        raise FGLError(rc, _lib.fgl_last_error().decode())
    return rc


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _prec(p) -> int:
    return PREC[p] if isinstance(p, str) else int(p)


# --- C-ABI mirrors -----------------------------------------------------------

def fgl_last_error() -> str:
    return _lib.fgl_last_error().decode()


def fgl_tune_cache(path) -> int:
    """Load tuned tiles from `path` (JSON lines) and write later tunings
    there; None stops writing."""
    return _check(_lib.fgl_tune_cache(None if path is None else os.fsencode(path)))


def fgl_model_create(K, freqs, data, nu_ref, N, F, T, t_cmb, flags=0):
    """Returns an opaque model handle; raises FGLError on failure."""
    K = np.ascontiguousarray(K, dtype=np.float32)
    freqs, data = _f64(freqs), _f64(data)
    h = _vp()
    _check(_lib.fgl_model_create(K.ctypes.data_as(_fp), freqs.ctypes.data_as(_dp),
                                 data.ctypes.data_as(_dp), float(nu_ref), int(N), int(F),
                                 int(T), float(t_cmb), int(flags), ctypes.byref(h)))
    return h


def fgl_model_create_masks(K, freqs, data, nu_ref, n_alpha, n_beta, F, T, t_cmb,
                           flags=0):
    """Amplitude masks crossed with spectral-index masks: K [n_alpha, n_beta,
    F, T]; returns an opaque model handle; raises FGLError on failure."""
    K = np.ascontiguousarray(K, dtype=np.float32)
    freqs, data = _f64(freqs), _f64(data)
    h = _vp()
    _check(_lib.fgl_model_create_masks(K.ctypes.data_as(_fp), freqs.ctypes.data_as(_dp),
                                       data.ctypes.data_as(_dp), float(nu_ref), int(n_alpha),
                                       int(n_beta), int(F), int(T), float(t_cmb), int(flags),
                                       ctypes.byref(h)))
    return h


def fgl_loglike_batch(model, theta, B, out, prec):
    return _check(_lib.fgl_loglike_batch(model, theta.ctypes.data_as(_dp), int(B),
                                         out.ctypes.data_as(_dp), _prec(prec)))


def fgl_loglike_batch_device(model, d_theta: int, B, d_out: int, prec, stream: int = 0):
    return _check(_lib.fgl_loglike_batch_device(model, _vp(d_theta), int(B), _vp(d_out),
                                                _prec(prec), _vp(stream)))


def fgl_loglike_batch_device_noalloc(model, d_theta: int, B, d_out: int, prec, stream: int = 0):
    return _check(_lib.fgl_loglike_batch_device_noalloc(model, _vp(d_theta), int(B), _vp(d_out),
                                                        _prec(prec), _vp(stream)))


def fgl_loglike_grad_batch(model, theta, B, out, grad, prec="fp64"):
    return _check(_lib.fgl_loglike_grad_batch(model, theta.ctypes.data_as(_dp), int(B),
                                              out.ctypes.data_as(_dp), grad.ctypes.data_as(_dp),
                                              _prec(prec)))


def fgl_loglike_grad_batch_device(model, d_theta: int, B, d_out: int, d_grad: int,
                                  prec="fp64", stream: int = 0):
    return _check(_lib.fgl_loglike_grad_batch_device(model, _vp(d_theta), int(B), _vp(d_out),
                                                     _vp(d_grad), _prec(prec), _vp(stream)))


def fgl_model_destroy(model):
    return _check(_lib.fgl_model_destroy(model))


def fgl_serve_create(budget_bytes: int, max_inflight: int):
    h = _vp()
    _check(_lib.fgl_serve_create(int(budget_bytes), int(max_inflight), ctypes.byref(h)))
    return h


def fgl_serve_submit(server, model, theta, B, out, prec) -> int:
    t = ctypes.c_uint64()
    _check(_lib.fgl_serve_submit(server, model, theta.ctypes.data_as(_dp), int(B),
                                 out.ctypes.data_as(_dp), _prec(prec), ctypes.byref(t)))
    return t.value


def fgl_serve_poll(server, ticket: int):
    """(done, latency_us); raises FGLError when the request failed."""
    d = ctypes.c_int()
    lat = ctypes.c_double()
    _check(_lib.fgl_serve_poll(server, ctypes.c_uint64(ticket), ctypes.byref(d),
                               ctypes.byref(lat)))
    return bool(d.value), lat.value


def fgl_serve_drain(server):
    return _check(_lib.fgl_serve_drain(server))


def fgl_serve_destroy(server):
    return _check(_lib.fgl_serve_destroy(server))


# --- convenience wrappers ------------------------------------------------------

class Model:
    """A resident model: K [N,F,T] (float32), freqs [F], data [F,T].

    With ``n_alpha`` > 0 the N = n_alpha * n_beta regions of K are amplitude
    masks crossed with spectral-index masks, region i * n_beta + j (K may
    also be given as [n_alpha, n_beta, F, T])."""

    def __init__(self, K, freqs, data, nu_ref: float = 230.0, t_cmb: float = 2.725,
                 flags: int = 0, n_alpha: int = 0):
        K = np.ascontiguousarray(K, dtype=np.float32)
        if K.ndim == 4:
            if n_alpha not in (0, K.shape[0]):
                raise ValueError("n_alpha disagrees with K's shape")
            n_alpha = K.shape[0]
            K = K.reshape(-1, K.shape[2], K.shape[3])
        if K.ndim != 3:
            raise ValueError("K must be [N, F, T] or [n_alpha, n_beta, F, T]")
        N, F, T = K.shape
        self.N, self.F, self.T = N, F, T
        self.flags = flags
        self.n_alpha = int(n_alpha)
        if n_alpha:
            if N % n_alpha:
                raise ValueError("N is not a multiple of n_alpha")
            self.handle = fgl_model_create_masks(K, freqs, data, nu_ref, n_alpha,
                                                 N // n_alpha, F, T, t_cmb, flags)
        else:
            self.handle = fgl_model_create(K, freqs, data, nu_ref, N, F, T, t_cmb, flags)
        self.P = _lib.fgl_model_nparams(self.handle)

    @classmethod
    def from_workload(cls, w, flags: int = 0) -> "Model":
        return cls(w.K, w.freqs, w.data, w.nu_ref, w.t_cmb, flags,
                   n_alpha=getattr(w, "n_alpha", 0))

    @property
    def form(self) -> str:
        """'direct', 'projected' or 'thin': the form of the mixed evaluation."""
        f = _lib.fgl_mixed_form(self.handle)
        return {FGL_FORM_PROJECTED: "projected", FGL_FORM_THIN: "thin"}.get(f, "direct")

    def loglike(self, theta, prec="mixed") -> np.ndarray:
        th = _f64(theta).reshape(-1, self.P)
        out = np.empty(th.shape[0], dtype=np.float64)
        fgl_loglike_batch(self.handle, th, th.shape[0], out, prec)
        return out

    def loglike_grad(self, theta, prec="fp64"):
        """(lnL [B], d lnL / d theta [B, P]) for host rows (FP64)."""
        th = _f64(theta).reshape(-1, self.P)
        out = np.empty(th.shape[0], dtype=np.float64)
        grad = np.empty_like(th)
        fgl_loglike_grad_batch(self.handle, th, th.shape[0], out, grad, prec)
        return out, grad

    def loglike_grad_device(self, theta, out=None, grad=None, prec="fp64", stream=None):
        """Device variant: theta a contiguous float64 CUDA tensor [B, P];
        returns (out [B], grad [B, P]) torch tensors, enqueued on `stream`."""
        import torch
        if theta.dtype != torch.float64 or not theta.is_cuda or not theta.is_contiguous():
            raise ValueError("theta must be a contiguous float64 device tensor")
        B = theta.shape[0]
        if out is None:
            out = torch.empty(B, dtype=torch.float64, device=theta.device)
        if grad is None:
            grad = torch.empty((B, self.P), dtype=torch.float64, device=theta.device)
        s = stream if stream is not None else torch.cuda.current_stream(theta.device)
        fgl_loglike_grad_batch_device(self.handle, theta.data_ptr(), B, out.data_ptr(),
                                      grad.data_ptr(), prec, s.cuda_stream)
        return out, grad

    def loglike_device(self, theta, out=None, prec="mixed", stream=None):
        """theta: torch float64 CUDA tensor [B, P]; returns out (torch, [B]),
        enqueued on `stream` (default: torch's current stream)."""
        import torch
        if theta.dtype != torch.float64 or not theta.is_cuda or not theta.is_contiguous():
            raise ValueError("theta must be a contiguous float64 device tensor")
        B = theta.shape[0]
        if out is None:
            out = torch.empty(B, dtype=torch.float64, device=theta.device)
        s = stream if stream is not None else torch.cuda.current_stream(theta.device)
        fgl_loglike_batch_device(self.handle, theta.data_ptr(), B, out.data_ptr(), prec,
                                 s.cuda_stream)
        return out

    def loglike_device_noalloc(self, theta, out, prec="mixed", stream=None):
        """As loglike_device, through the entry point that allocates
        nothing (out must be given: a float64 device tensor [B])."""
        import torch
        if theta.dtype != torch.float64 or not theta.is_cuda or not theta.is_contiguous():
            raise ValueError("theta must be a contiguous float64 device tensor")
        if out.dtype != torch.float64 or not out.is_cuda or out.numel() < theta.shape[0]:
            raise ValueError("out must be a float64 device tensor of at least B values")
        s = stream if stream is not None else torch.cuda.current_stream(theta.device)
        fgl_loglike_batch_device_noalloc(self.handle, theta.data_ptr(), theta.shape[0],
                                         out.data_ptr(), prec, s.cuda_stream)
        return out

    def tune(self, B: int, prec="mixed"):
        _check(_lib.fgl_tune(self.handle, int(B), _prec(prec)))

    def set_tile(self, B: int, prec, waves: int, chans: int, occupancy: int = 2):
        _check(_lib.fgl_set_tile(self.handle, int(B), _prec(prec), int(waves), int(chans),
                                 int(occupancy)))

    def tile(self, B: int, prec="mixed"):
        """(waves per workgroup, channels per workgroup, waves per SIMD)."""
        w, c, p = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(_lib.fgl_get_tile(self.handle, int(B), _prec(prec), ctypes.byref(w),
                                 ctypes.byref(c), ctypes.byref(p)))
        return w.value, c.value, p.value

    def kernel_timing(self, enable: bool = True, every: int = 1):
        """Record the likelihood kernel's duration on every `every`-th call
        (from now on, counters reset) or stop recording."""
        _check(_lib.fgl_kernel_timing(self.handle, int(every) if enable else 0))

    def kernel_time(self):
        """(summed likelihood-kernel milliseconds, launches) since the last
        kernel_timing(True)."""
        ms, n = ctypes.c_double(), ctypes.c_int64()
        _check(_lib.fgl_kernel_time(self.handle, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    @property
    def nbytes(self) -> int:
        return int(_lib.fgl_model_bytes(self.handle))

    def close(self):
        if self.handle is not None:
            fgl_model_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            if self.handle is not None:
                _lib.fgl_model_destroy(self.handle)
        except Exception:
            pass


class Server:
    """Continuous-batching server over resident models."""

    def __init__(self, budget_bytes: int = 0, max_inflight: int = 8):
        self.handle = fgl_serve_create(budget_bytes, max_inflight)
        self._keep = {}

    def submit(self, model: Model, theta, prec="mixed"):
        th = _f64(theta).reshape(-1, model.P)
        out = np.empty(th.shape[0], dtype=np.float64)
        t = fgl_serve_submit(self.handle, model.handle, th, th.shape[0], out, prec)
        self._keep[t] = (th, out)
        return t

    def poll(self, ticket: int):
        """None while running; (out, latency_us) when done."""
        try:
            done, lat = fgl_serve_poll(self.handle, ticket)
        except FGLError:
            self._keep.pop(ticket, None)
            raise
        if not done:
            return None
        _, out = self._keep.pop(ticket)
        return out, lat

    def drain(self):
        fgl_serve_drain(self.handle)

    def cancel(self, ticket: int):
        """Cancel a queued request (its poll then raises FGL_ECANCELED);
        FGLError(FGL_EBUSY) once it is launched or complete."""
        _check(_lib.fgl_serve_cancel(self.handle, ctypes.c_uint64(ticket)))

    def set_timeout(self, max_wait_us: float):
        """Requests queued longer than this (microseconds; 0: no limit)
        complete with FGL_ETIMEDOUT."""
        _check(_lib.fgl_serve_set_timeout(self.handle, float(max_wait_us)))

    def hold(self, on: bool = True):
        """Hold admission (requests only queue) or release it (the queue is
        then planned at once: merged per model, shared across models)."""
        _check(_lib.fgl_serve_hold(self.handle, 1 if on else 0))

    def set_sharing(self, max_models_per_launch: int):
        """Up to this many models of one kernel variant per launch (1: off)."""
        _check(_lib.fgl_serve_set_sharing(self.handle, int(max_models_per_launch)))

    def stats(self):
        """(launches, shared launches, model groups in shared launches)."""
        a, b, c = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
        _check(_lib.fgl_serve_stats(self.handle, ctypes.byref(a), ctypes.byref(b),
                                    ctypes.byref(c)))
        return a.value, b.value, c.value

    def close(self):
        if self.handle is not None:
            fgl_serve_destroy(self.handle)
            self.handle = None


class Chains:
    """Slice-sampling chains on the device for a resident model
    (fgl_chains_*): the replacement step of batched nested sampling."""

    def __init__(self, model: Model, max_chains: int, lo, hi, seed: int = 0):
        lo, hi = _f64(lo), _f64(hi)
        if lo.size != model.P or hi.size != model.P:
            raise ValueError("lo and hi need one entry per parameter")
        h = _vp()
        _check(_lib.fgl_chains_create(model.handle, int(max_chains), lo.ctypes.data_as(_dp),
                                      hi.ctypes.data_as(_dp), ctypes.c_uint64(seed),
                                      ctypes.byref(h)))
        self.handle = h
        self.model = model
        self.P = model.P

    def run(self, x0, l0, lstar: float, chol, steps: int, prec="mixed"):
        """(x [n, P], lnL [n], in-box evaluations, rounds) after `steps` slice
        steps of each chain from x0 under lnL > lstar."""
        x0 = _f64(x0).reshape(-1, self.P)
        l0 = _f64(l0)
        chol = _f64(chol).reshape(self.P, self.P)
        n = x0.shape[0]
        x = np.empty_like(x0)
        lx = np.empty(n)
        ev, rounds = ctypes.c_int64(), ctypes.c_int64()
        _check(_lib.fgl_chains_run(self.handle, x0.ctypes.data_as(_dp), l0.ctypes.data_as(_dp),
                                   n, float(lstar), chol.ctypes.data_as(_dp), int(steps),
                                   _prec(prec), x.ctypes.data_as(_dp), lx.ctypes.data_as(_dp),
                                   ctypes.byref(ev), ctypes.byref(rounds)))
        return x, lx, ev.value, rounds.value

    def close(self):
        if self.handle is not None:
            _check(_lib.fgl_chains_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            if self.handle is not None:
                _lib.fgl_chains_destroy(self.handle)
        except Exception:
            pass


# --- region construction -------------------------------------------------------

WEIGHTS = {"horizon": 0, "sky": 1, "beam": 2}
PARTITIONS = {"hierarchical": 0, "recursive": 1}


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.int32)


def fgl_partition(beta, weight, n_regions: int, method="recursive") -> np.ndarray:
    """Edges [n_regions + 1] of Alg. method1 / method2 on the weighted CDF
    (host computation in the library)."""
    b, w = _f64(beta).ravel(), _f64(weight).ravel()
    if b.size != w.size:
        raise ValueError("beta and weight differ in size")
    edges = np.empty(int(n_regions) + 1, dtype=np.float64)
    m = PARTITIONS[method] if isinstance(method, str) else int(method)
    _check(_lib.fgl_partition(b.ctypes.data_as(_dp), w.ctypes.data_as(_dp), b.size,
                              int(n_regions), m, edges.ctypes.data_as(_dp)))
    return edges


class SkyModel:
    """A resident sky for region construction: maps as in workload.sky.Sky
    (omega [nlat], t_ex / beta [nlat, nlon], beam [F, nlat, nlon] FP32,
    horizon [nlat, nlon], freqs [F])."""

    def __init__(self, omega, t_ex, beta, beam, horizon, freqs, nu0=230.0, t_cmb=2.725):
        self._keep = (_f64(omega), _f64(t_ex), _f64(beta),
                      np.ascontiguousarray(beam, dtype=np.float32),
                      np.ascontiguousarray(horizon, dtype=np.uint8), _f64(freqs))
        om, tx, bt, bm, hz, fr = self._keep
        self.nlat, self.nlon = tx.shape
        self.F = fr.size
        h = _vp()
        _check(_lib.fgl_sky_create(self.nlat, self.nlon, self.F, om.ctypes.data_as(_dp),
                                   tx.ctypes.data_as(_dp), bt.ctypes.data_as(_dp),
                                   bm.ctypes.data_as(_fp),
                                   hz.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                   fr.ctypes.data_as(_dp), float(nu0), float(t_cmb),
                                   ctypes.byref(h)))
        self.handle = h
        self._keep = None

    @classmethod
    def from_sky(cls, s) -> "SkyModel":
        return cls(s.omega, s.t_ex, s.beta, s.beam, s.horizon, s.freqs, s.nu0, s.t_cmb)

    def importance(self, shifts, scheme="beam") -> np.ndarray:
        sh = _i32(shifts)
        out = np.empty((self.nlat, self.nlon), dtype=np.float64)
        sc = WEIGHTS[scheme] if isinstance(scheme, str) else int(scheme)
        _check(_lib.fgl_sky_importance(self.handle, sh.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                       sh.size, sc, out.ctypes.data_as(_dp)))
        return out

    def chromatic(self, edges, shifts) -> np.ndarray:
        e, sh = _f64(edges), _i32(shifts)
        N = e.size - 1
        K = np.empty((N, self.F, sh.size), dtype=np.float64)
        _check(_lib.fgl_sky_chromatic(self.handle, e.ctypes.data_as(_dp), N,
                                      sh.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), sh.size,
                                      K.ctypes.data_as(_dp)))
        return K

    def kernel_ms(self) -> float:
        ms = ctypes.c_double()
        _check(_lib.fgl_sky_kernel_ms(self.handle, ctypes.byref(ms)))
        return ms.value

    def close(self):
        if self.handle is not None:
            _check(_lib.fgl_sky_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            if self.handle is not None:
                _lib.fgl_sky_destroy(self.handle)
        except Exception:
            pass


def fgl_noise_loglike(n: int, R: int, sigma_noise: float, sigma_like: float,
                      seed: int = 0, timed: bool = False):
    """lnL [R] of noise-only data sets of n residuals (accuracy criterion,
    Sec. 5); with timed=True also the kernel's duration in ms."""
    out = np.empty(int(R), dtype=np.float64)
    ms = ctypes.c_double(0.0)
    _check(_lib.fgl_noise_loglike(int(n), int(R), float(sigma_noise), float(sigma_like),
                                  int(seed) & 0xFFFFFFFFFFFFFFFF, out.ctypes.data_as(_dp),
                                  ctypes.byref(ms) if timed else None))
    return (out, ms.value) if timed else out


def fgl_chains_philox(ctr, k0: int, k1: int) -> np.ndarray:
    """Philox4x32-10 blocks [n, 4] of counter blocks ctr [n, 4] (uint32)
    under the key (k0, k1), by the device generator of the chains."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    out = np.empty_like(c)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    _check(_lib.fgl_chains_philox(c.ctypes.data_as(u32p), c.shape[0], int(k0) & 0xFFFFFFFF,
                                  int(k1) & 0xFFFFFFFF, out.ctypes.data_as(u32p)))
    return out


def fgl_noise_quantile(lnl_noise, lbar) -> np.ndarray:
    """q = fraction of lnl_noise at or below each lbar (computed on the device)."""
    ref, lb = _f64(lnl_noise).ravel(), _f64(lbar).ravel()
    q = np.empty(lb.size, dtype=np.float64)
    _check(_lib.fgl_noise_quantile(ref.ctypes.data_as(_dp), ref.size, lb.ctypes.data_as(_dp),
                                   lb.size, q.ctypes.data_as(_dp)))
    return q
