"""Launch machinery on the GPU: hipGraph replay of the device-pointer call
(FGL_DEVICE_GRAPHS=1) and the persisted tuner cache.

Graph replays must give bitwise the eager result (the first sighting of a
call runs eagerly, the second is captured, later ones replay), also with
other models' work and buffers in between.  The tuner cache must hand a
measured tile to a new model of the same shape, in this process and in a
new one that names the same file.
"""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

import workload
from tests.gpu_util import lib, say

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_device_call_graph_replays_bitwise(monkeypatch):
    import torch
    fgl = lib()
    torch.cuda.set_device(0)
    w = workload.config(workload.HEADLINE, B=2048, batch="mixed")
    other = workload.config(workload.MEDIUM, B=1000, batch="mixed")
    monkeypatch.setenv("FGL_DEVICE_GRAPHS", "1")     # read when a model is created
    m = fgl.Model.from_workload(w)
    mo = fgl.Model.from_workload(other)
    monkeypatch.delenv("FGL_DEVICE_GRAPHS")
    th = torch.from_numpy(w.theta).cuda()
    tho = torch.from_numpy(other.theta).cuda()
    for prec in ("mixed", "fp32", "fp64"):
        ref = m.loglike(w.theta, prec)           # host call (eager or its own graph)
        out = torch.empty(w.B, dtype=torch.float64, device="cuda")
        for call in range(6):                    # eager, capture, replays
            out.fill_(np.nan)
            m.loglike_device(th, out, prec)
            mo.loglike_device(tho, prec=prec)    # other work in between
            torch.cuda.synchronize()
            got = out.cpu().numpy()
            assert np.array_equal(got, ref), (prec, call)
        # a second output buffer is another graph; a side stream too
        out2 = torch.empty(w.B, dtype=torch.float64, device="cuda")
        s = torch.cuda.Stream()
        for call in range(3):
            with torch.cuda.stream(s):
                m.loglike_device(th, out2, prec, stream=s)
            s.synchronize()
            assert np.array_equal(out2.cpu().numpy(), ref), (prec, "side stream", call)
        say(f"  graph replays {prec}: bitwise equal to the eager call")
    m.close()
    mo.close()


def test_tuner_cache_persists(tmp_path):
    import torch
    fgl = lib()
    torch.cuda.set_device(0)
    path = str(tmp_path / "tiles.jsonl")
    fgl.fgl_tune_cache(path)
    try:
        w = workload.config(workload.HEADLINE, B=4096)
        m = fgl.Model.from_workload(w)
        m.tune(w.B, "mixed")
        tuned = m.tile(w.B, "mixed")
        m.close()
        lines = [json.loads(x) for x in open(path) if x.strip()]
        hit = [e for e in lines if e["N"] == 32 and e["T"] == 96 and e["bucket"] == 4096
               and e["kind"] == 0]
        assert hit and (hit[-1]["waves"], hit[-1]["fc"], hit[-1]["occ"]) == tuned, (lines, tuned)
        assert hit[-1]["arch"].startswith("gfx950")
        # a new model of the same shape starts from the cached tile
        m2 = fgl.Model.from_workload(w)
        assert m2.tile(w.B, "mixed") == tuned
        m2.close()
        # so does a new process that names the file
        code = ("import sys; sys.path.insert(0, %r)\n"
                "import workload\nfrom paper_2603_13196_amd import fgl\n"
                "w = workload.config(workload.HEADLINE, B=4096)\n"
                "m = fgl.Model.from_workload(w)\nprint(*m.tile(w.B, 'mixed'))\n" % ROOT)
        env = dict(os.environ, FGL_TUNE_CACHE=path)
        p = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True,
                           text=True, timeout=120)
        assert p.returncode == 0, p.stderr[-2000:]
        got = tuple(int(x) for x in p.stdout.split()[-3:])
        say(f"  tuned {tuned}, new process read {got}")
        assert got == tuned
    finally:
        fgl.fgl_tune_cache(None)
