"""The allocation-free device entry point against fgl_loglike_batch_device.

fgl_loglike_batch_device_noalloc runs the same kernels on a workspace in a
fixed device array: its results must be bitwise those of the allocating
device call, on two calls in a row (the second with a smaller batch, so the
array holds the first call's contents), in every precision and form; a
batch beyond the array is refused with FGL_EINVAL.
"""
import numpy as np
import pytest

import workload
from tests.gpu_util import lib, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kind", ["headline", "direct", "masks", "thin"])
def test_noalloc_matches_device_call(kind):
    import torch
    fgl = lib()
    torch.cuda.set_device(0)
    if kind == "masks":
        w = workload.make_masks(2, 16, workload.freq_grid(50.0, 200.0, 0.5), 96, 4096,
                                workload.SEED_BASE + 5, batch="mixed")
        flags = 0
    elif kind == "thin":
        w = workload.config(workload.MEDIUM, B=4096, batch="mixed")
        flags = 0
    else:
        w = workload.config(workload.HEADLINE, B=4096, batch="mixed")
        flags = fgl.FGL_MIXED_DIRECT if kind == "direct" else 0
    m = fgl.Model.from_workload(w, flags)
    say(f"noalloc {kind}: N={w.N} F={w.F} T={w.T} form={m.form}")
    th = torch.from_numpy(w.theta).cuda()
    for prec in ("mixed", "fp32", "fp64"):
        for B in (4096, 1000):           # second call smaller: stale contents
            ref = m.loglike_device(th[:B].contiguous(), prec=prec)
            out = torch.full((B,), np.nan, dtype=torch.float64, device="cuda")
            m.loglike_device_noalloc(th[:B].contiguous(), out, prec=prec)
            torch.cuda.synchronize()
            a, b = out.cpu().numpy(), ref.cpu().numpy()
            say(f"  {prec} B={B}: equal={np.array_equal(a, b)}")
            assert np.array_equal(a, b), (kind, prec, B)
    m.close()


def test_noalloc_refuses_oversized_batch():
    import torch
    fgl = lib()
    torch.cuda.set_device(0)
    w = workload.config(workload.HEADLINE, B=256)
    m = fgl.Model.from_workload(w)
    B = 1 << 17                          # 131072 rows need ~120 MB of workspace
    th = torch.zeros((B, w.P), dtype=torch.float64, device="cuda")
    out = torch.zeros(B, dtype=torch.float64, device="cuda")
    with pytest.raises(fgl.FGLError) as ei:
        m.loglike_device_noalloc(th, out)
    assert ei.value.code == fgl.FGL_EINVAL
    say(f"  refused: {ei.value}")
    m.close()
