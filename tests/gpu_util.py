"""Helpers shared by the GPU tests: library/oracle loading and the parity bar.

Tolerances (from the statement of the path):
  mixed precision   |dlnL| <= 1e-6 |lnL_oracle| + 1e-3
  plain FP64        |dlnL| <= 1e-9 |lnL_oracle|, except on rows where the
                    chi-square term and the normalisation cancel to less
                    than a tenth of their magnitude S (there lnL is near
                    zero and no FP64 evaluation resolves 1e-9 of it): 1e-9 S
  plain FP32        measured and reported; asserted only against a loose
                    bound on prior draws (an FP32 model cannot meet the
                    mixed bound near the posterior peak).

With FGL_MARGIN_LOG set to a path, every check appends one JSON line (case,
precision, rows, max |dlnL|, max and 99th percentile of |dlnL|/tolerance)
to that file; tests/margin_table.py prints the collected record.
"""
from __future__ import annotations

import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def lib():
    """The binding; builds the library only when it is missing."""
    from paper_2603_13196_amd import LIB_PATH
    if not os.path.exists(LIB_PATH):
        from paper_2603_13196_amd import build
        build.build()
    from paper_2603_13196_amd import fgl
    return fgl


def thin_form(N: int, T: int) -> bool:
    """Whether the library evaluates a model per row in FP64 (its thin
    form): N <= 32, T <= 64 and the cost rule documented with
    FGL_FORM_THIN in include/fgl.h."""
    slots = next((s for s in (4, 8, 12, 16, 24, 32) if N <= s), None)
    if slots is None or T > 64:
        return False
    scale = {24: 117, 32: 90, 12: 97}.get(slots, 100)
    return (slots * T + 12 * slots + 2 * T) * scale <= (650 if T <= 32 else 580) * 100


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def tol_mixed(ref):
    return 1e-6 * np.abs(ref) + 1e-3


def tol_fp64(ref, scale=None):
    """1e-9 |lnL|; where the chi-square term and the normalisation cancel
    to less than a tenth of their magnitude S (given as ``scale``), 1e-9 S."""
    a = np.abs(ref)
    if scale is None:
        return 1e-9 * a
    s = np.asarray(scale)
    return 1e-9 * np.where(a >= 0.1 * s, a, s)


def record(label: str, kind: str, d, t) -> None:
    """Append a case's margin to the record named by FGL_MARGIN_LOG."""
    path = os.environ.get("FGL_MARGIN_LOG")
    if not path:
        return
    d = np.asarray(d, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    r = d / t if d.size else np.zeros(1)
    rec = {"case": label, "prec": kind, "rows": int(d.size),
           "max_abs": float(d.max()) if d.size else 0.0,
           "max_ratio": float(r.max()), "p99_ratio": float(np.percentile(r, 99))}
    with open(path, "a") as f:
        f.write(json.dumps(rec) + "\n")


def term_scale(ref, sigma, n):
    """|chi2/(2 sigma^2)| + |n/2 ln(2 pi sigma^2)| recovered from lnL."""
    norm = -0.5 * n * np.log(2.0 * np.pi * np.asarray(sigma) ** 2)
    return np.abs(ref - norm) + np.abs(norm)


def check(got, ref, kind: str, label: str = "", theta=None, n=None):
    """Element-wise parity; infinities must match exactly.  For FP64 the
    bound is relative to the magnitude of lnL's terms, computed from the
    rows' sigma (last column of theta) and n = F T when they are given."""
    got = np.asarray(got)
    ref = np.asarray(ref)
    scale = None
    if theta is not None and n is not None:
        sig = np.asarray(theta)[:, -1]
        with np.errstate(all="ignore"):
            scale = term_scale(ref, np.where(sig > 0, sig, 1.0), n)
    assert got.shape == ref.shape
    inf = ~np.isfinite(ref)
    assert np.array_equal(got[inf], ref[inf]), f"{label}: non-finite rows differ"
    g, r = got[~inf], ref[~inf]
    sc = None if scale is None else np.asarray(scale)[~inf]
    assert np.all(np.isfinite(g)), f"{label}: GPU gave non-finite values on valid rows"
    d = np.abs(g - r)
    if kind == "mixed":
        t = tol_mixed(r)
    elif kind == "fp64":
        t = tol_fp64(r, sc)
    elif kind == "fp32":
        t = 1e-4 * np.abs(r) + 1e-3
    else:
        raise ValueError(kind)
    worst = int(np.argmax(d / t)) if d.size else 0
    say(f"  {label} {kind}: rows={d.size} max|d|={d.max() if d.size else 0:.3e} "
        f"max|d|/tol={(d / t).max() if d.size else 0:.3e}")
    record(label, kind, d, t)
    assert np.all(d <= t), (f"{label} {kind}: row {worst} |d|={d[worst]:.4e} "
                            f"tol={t[worst]:.4e} ref={r[worst]:.6e}")
    return d
