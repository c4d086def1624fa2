"""Profiling ranges: with FGL_ROCTX=1 the library's calls push roctx ranges
that rocprofv3 --marker-trace records, named for the call with its sizes; a
likelihood call's kernels run inside its range."""
import csv
import glob
import os
import shutil
import subprocess
import sys
import tempfile

import pytest

from tests.gpu_util import say

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import numpy as np, torch
import workload
from paper_2603_13196_amd import fgl
w = workload.config(workload.SMALL, B=300)
m = fgl.Model.from_workload(w)
m.loglike(w.theta, "mixed")
th = torch.from_numpy(w.theta).cuda()
m.loglike_device(th, prec="fp64")
torch.cuda.synchronize()
srv = fgl.Server(max_inflight=1)
t = srv.submit(m, w.theta[:100])
srv.drain()
srv.poll(t)
srv.close()
m.close()
print("script ok", flush=True)
"""


def test_roctx_ranges_in_marker_trace():
    prof = shutil.which("rocprofv3")
    if prof is None:
        pytest.skip("rocprofv3 is not on PATH")
    out = tempfile.mkdtemp(prefix="fgl_roctx_", dir="/tmp")
    env = dict(os.environ, FGL_ROCTX="1", TMPDIR="/tmp", PYTHONPATH=ROOT)
    cmd = [prof, "--marker-trace", "--kernel-trace", "--output-format", "csv", "-d", out,
           "-o", "run", "--", sys.executable, "-c", SCRIPT]
    say("running " + " ".join(cmd[:8]) + " ...")
    p = subprocess.run(cmd, cwd="/tmp", env=env, capture_output=True, text=True, timeout=300)
    assert "script ok" in p.stdout, (p.returncode, p.stdout[-2000:], p.stderr[-4000:])
    markers = glob.glob(os.path.join(out, "**", "*marker*trace*.csv"), recursive=True)
    kernels = glob.glob(os.path.join(out, "**", "*kernel_trace*.csv"), recursive=True)
    assert markers and kernels, os.listdir(out)
    rows = list(csv.DictReader(open(markers[0])))
    names = [r.get("Function") or r.get("Message") or r.get("Name") or "" for r in rows]
    say(f"  {len(rows)} marker records: {sorted(set(names))[:12]}")
    want = ["fgl_model_create N=", "fgl_loglike_batch prec=0 B=300",
            "fgl_loglike_batch_device prec=2 B=300", "serve launch: 1 requests, 100 rows"]
    for wnt in want:
        assert any(n.startswith(wnt) for n in names), (wnt, names)
    # the host call's likelihood kernels run inside its range
    rng = next(r for r, n in zip(rows, names) if n.startswith("fgl_loglike_batch prec=0"))
    t0, t1 = int(rng["Start_Timestamp"]), int(rng["End_Timestamp"])
    ks = [r for r in csv.DictReader(open(kernels[0]))
          if "k_" in r["Kernel_Name"] and t0 <= int(r["Start_Timestamp"]) <= t1]
    say(f"  kernels inside the host call's range: {sorted(set(r['Kernel_Name'].split('(')[0] for r in ks))}")
    assert any("k_prep" in r["Kernel_Name"] for r in ks)
    shutil.rmtree(out, ignore_errors=True)
