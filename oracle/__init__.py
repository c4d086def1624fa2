"""ctypes wrapper of the FP64 CPU oracle (``fgl_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the library.  The oracle is built with
gcc from its own single C file; it shares nothing with the HIP library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "fgl_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
NO_21CM = 1

CFLAGS = ["-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
          "-fno-fast-math", "-std=c11", "-D_DEFAULT_SOURCE"]


def build(src: str = SRC, out: str = LIB,
          extra: Sequence[str] = ()) -> str:
    """Compile the oracle (or a planted-mistake variant of it) with gcc."""
    tmp = out + ".tmp%d" % os.getpid()
    cmd = ["gcc", *CFLAGS, *extra, src, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    os.replace(tmp, out)
    return out


class Oracle:
    def __init__(self, path: str):
        self.path = path
        lib = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        fp = ctypes.POINTER(ctypes.c_float)
        lib.oracle_loglike.argtypes = [fp, dp, dp, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_int,
                                       ctypes.c_int, ctypes.c_int,
                                       ctypes.c_uint, dp, ctypes.c_int, dp,
                                       ctypes.c_int]
        lib.oracle_loglike.restype = ctypes.c_int
        lib.oracle_model.argtypes = [fp, dp, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_uint, dp, dp]
        lib.oracle_model.restype = ctypes.c_int
        lib.oracle_loglike_masks.argtypes = [fp, dp, dp, ctypes.c_double,
                                             ctypes.c_double, ctypes.c_int,
                                             ctypes.c_int, ctypes.c_int,
                                             ctypes.c_int, ctypes.c_uint, dp,
                                             ctypes.c_int, dp, ctypes.c_int]
        lib.oracle_loglike_masks.restype = ctypes.c_int
        lib.oracle_model_masks.argtypes = [fp, dp, ctypes.c_double,
                                           ctypes.c_double, ctypes.c_int,
                                           ctypes.c_int, ctypes.c_int,
                                           ctypes.c_int, ctypes.c_uint, dp, dp]
        lib.oracle_model_masks.restype = ctypes.c_int
        lib.oracle_grad_batch_masks.argtypes = [fp, dp, dp, ctypes.c_double,
                                                ctypes.c_double, ctypes.c_int,
                                                ctypes.c_int, ctypes.c_int,
                                                ctypes.c_int, ctypes.c_uint, dp,
                                                ctypes.c_int, dp, dp, ctypes.c_int]
        lib.oracle_grad_batch_masks.restype = ctypes.c_int
        lib.oracle_max_threads.restype = ctypes.c_int
        self._lib = lib

    @staticmethod
    def _f64(a):
        return np.ascontiguousarray(a, dtype=np.float64)

    def loglike(self, K, freqs, data, nu_ref, t_cmb, theta, flags: int = 0,
                threads: int = 0) -> np.ndarray:
        K = np.ascontiguousarray(K, dtype=np.float32)
        freqs, data, theta = self._f64(freqs), self._f64(data), self._f64(theta)
        N, F, T = K.shape
        theta = theta.reshape(-1, theta.shape[-1])
        B = theta.shape[0]
        out = np.empty(B, dtype=np.float64)
        dp = ctypes.POINTER(ctypes.c_double)
        rc = self._lib.oracle_loglike(
            K.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
            freqs.ctypes.data_as(dp), data.ctypes.data_as(dp),
            float(nu_ref), float(t_cmb), N, F, T, flags,
            theta.ctypes.data_as(dp), B, out.ctypes.data_as(dp), int(threads))
        if rc != 0:
            raise RuntimeError(f"oracle_loglike failed ({rc})")
        return out

    def model(self, K, freqs, nu_ref, t_cmb, theta_row,
              flags: int = 0) -> Optional[np.ndarray]:
        K = np.ascontiguousarray(K, dtype=np.float32)
        freqs, th = self._f64(freqs), self._f64(theta_row)
        N, F, T = K.shape
        m = np.empty((F, T), dtype=np.float64)
        dp = ctypes.POINTER(ctypes.c_double)
        rc = self._lib.oracle_model(
            K.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
            freqs.ctypes.data_as(dp), float(nu_ref), float(t_cmb), N, F, T,
            flags, th.ctypes.data_as(dp), m.ctypes.data_as(dp))
        return m if rc == 0 else None

    def loglike_masks(self, K, freqs, data, nu_ref, t_cmb, theta,
                      flags: int = 0, threads: int = 0) -> np.ndarray:
        """Amplitude masks crossed with spectral-index masks:
        K [n_alpha, n_beta, F, T]; rows [beta.., alpha.., A, nu21, w, sigma]."""
        K = np.ascontiguousarray(K, dtype=np.float32)
        freqs, data, theta = self._f64(freqs), self._f64(data), self._f64(theta)
        NA, NB, F, T = K.shape
        theta = theta.reshape(-1, theta.shape[-1])
        B = theta.shape[0]
        out = np.empty(B, dtype=np.float64)
        dp = ctypes.POINTER(ctypes.c_double)
        rc = self._lib.oracle_loglike_masks(
            K.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
            freqs.ctypes.data_as(dp), data.ctypes.data_as(dp),
            float(nu_ref), float(t_cmb), NA, NB, F, T, flags,
            theta.ctypes.data_as(dp), B, out.ctypes.data_as(dp), int(threads))
        if rc != 0:
            raise RuntimeError(f"oracle_loglike_masks failed ({rc})")
        return out

    def model_masks(self, K, freqs, nu_ref, t_cmb, theta_row,
                    flags: int = 0) -> Optional[np.ndarray]:
        K = np.ascontiguousarray(K, dtype=np.float32)
        freqs, th = self._f64(freqs), self._f64(theta_row)
        NA, NB, F, T = K.shape
        m = np.empty((F, T), dtype=np.float64)
        dp = ctypes.POINTER(ctypes.c_double)
        rc = self._lib.oracle_model_masks(
            K.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
            freqs.ctypes.data_as(dp), float(nu_ref), float(t_cmb), NA, NB, F, T,
            flags, th.ctypes.data_as(dp), m.ctypes.data_as(dp))
        return m if rc == 0 else None

    def grad(self, K, freqs, data, nu_ref, t_cmb, theta, flags: int = 0,
             n_alpha: int = 0, threads: int = 0):
        """(lnL [B], d lnL / d theta [B, P]) of the spectral-index-only model
        (K [N, F, T], n_alpha = 0) or of the crossed-mask model (K
        [n_alpha, n_beta, F, T] or [n_alpha * n_beta, F, T])."""
        K = np.ascontiguousarray(K, dtype=np.float32)
        freqs, data, theta = self._f64(freqs), self._f64(data), self._f64(theta)
        F, T = K.shape[-2], K.shape[-1]
        N = int(np.prod(K.shape[:-2]))
        NA = n_alpha if K.ndim == 3 else K.shape[0]
        NB = N // max(NA, 1)
        theta = theta.reshape(-1, theta.shape[-1])
        B, P = theta.shape
        out = np.empty(B, dtype=np.float64)
        grad = np.empty((B, P), dtype=np.float64)
        dp = ctypes.POINTER(ctypes.c_double)
        rc = self._lib.oracle_grad_batch_masks(
            K.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
            freqs.ctypes.data_as(dp), data.ctypes.data_as(dp),
            float(nu_ref), float(t_cmb), NA, NB, F, T, flags,
            theta.ctypes.data_as(dp), B, out.ctypes.data_as(dp),
            grad.ctypes.data_as(dp), int(threads))
        if rc != 0:
            raise RuntimeError(f"oracle_grad_batch_masks failed ({rc})")
        return out, grad

    def grad_w(self, w, theta=None, threads: int = 0):
        th = w.theta if theta is None else theta
        return self.grad(w.K, w.freqs, w.data, w.nu_ref, w.t_cmb, th,
                         n_alpha=getattr(w, "n_alpha", 0), threads=threads)

    def max_threads(self) -> int:
        return int(self._lib.oracle_max_threads())

    # convenience on a workload object
    def loglike_w(self, w, theta=None, threads: int = 0) -> np.ndarray:
        th = w.theta if theta is None else theta
        na = getattr(w, "n_alpha", 0)
        if na:
            K4 = w.K.reshape(na, w.N // na, w.F, w.T)
            return self.loglike_masks(K4, w.freqs, w.data, w.nu_ref, w.t_cmb,
                                      th, threads=threads)
        return self.loglike(w.K, w.freqs, w.data, w.nu_ref, w.t_cmb, th,
                            threads=threads)


_cached: Optional[Oracle] = None


def load(rebuild: bool = False) -> Oracle:
    """Load the oracle, compiling it first when it is missing or older than
    its source."""
    global _cached
    if _cached is not None and not rebuild:
        return _cached
    stale = (not os.path.exists(LIB) or
             os.path.getmtime(LIB) < os.path.getmtime(SRC))
    if rebuild or stale:
        build()
    _cached = Oracle(LIB)
    return _cached
