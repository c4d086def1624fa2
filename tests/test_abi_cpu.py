"""CPU-side checks of the C-ABI library: it builds, loads, and exports every
symbol include/fgl.h declares; the binding refuses to work without it; the
product path never touches the oracle.  No likelihood is computed here."""
import os
import re
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fgl.h")
PKG = os.path.join(ROOT, "paper_2603_13196_amd")


def header_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(fgl_\w+)\s*\(", txt)))


@pytest.fixture(scope="module")
def libpath():
    from paper_2603_13196_amd import LIB_PATH
    if not os.path.exists(LIB_PATH):
        from paper_2603_13196_amd import build
        build.build()
    return LIB_PATH


def test_header_declares_the_boundary():
    fns = header_functions()
    for need in ("fgl_model_create", "fgl_loglike_batch", "fgl_loglike_batch_device",
                 "fgl_serve_create", "fgl_serve_submit", "fgl_serve_poll",
                 "fgl_serve_destroy", "fgl_model_destroy", "fgl_last_error"):
        assert need in fns


def test_library_exports_every_declared_symbol(libpath):
    out = subprocess.run(["nm", "-D", "--defined-only", libpath], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\sT\s(fgl_\w+)", out))
    missing = [f for f in header_functions() if f not in exported]
    assert not missing, missing


def test_binding_covers_every_symbol(libpath):
    from paper_2603_13196_amd import fgl
    assert set(header_functions()) <= set(fgl.EXPORTED)
    for f in header_functions():
        assert hasattr(fgl._lib, f)


def test_last_error_without_device_call(libpath):
    from paper_2603_13196_amd import fgl
    # argument validation happens before any device call
    with pytest.raises(fgl.FGLError) as e:
        fgl.fgl_model_create([[[1.0]]], [100.0], [[1.0]], 230.0, 0, 1, 1, 2.725)
    assert e.value.code == fgl.FGL_EINVAL
    assert "N=0" in fgl.fgl_last_error()
    K = [[[[1.0]]]]
    for na, nb, what in ((0, 1, "n_alpha=0"), (1, 0, "n_beta=0"), (2, 65, "128 regions")):
        with pytest.raises(fgl.FGLError) as e:
            fgl.fgl_model_create_masks(K, [100.0], [[1.0]], 230.0, na, nb, 1, 1, 2.725)
        assert e.value.code == fgl.FGL_EINVAL
        assert what in fgl.fgl_last_error(), fgl.fgl_last_error()


@pytest.mark.parametrize("args", [
    (0, 1, 0.025, 0.025), (2**31 + 1, 1, 0.025, 0.025), (2**30, 1025, 0.025, 0.025),
    (4, 0, 0.025, 0.025),
    (4, 2**23 + 1, 0.025, 0.025), (4, 1, -1.0, 0.025), (4, 1, 0.025, 0.0),
    (4, 1, float("nan"), 0.025), (4, 1, 0.025, float("inf")),
])
def test_noise_entry_rejects_bad_arguments(libpath, args):
    from paper_2603_13196_amd import fgl
    with pytest.raises(fgl.FGLError) as e:
        fgl.fgl_noise_loglike(*args)
    assert e.value.code == fgl.FGL_EINVAL
    for ref, lbar in (([], [1.0]), ([1.0], [])):
        with pytest.raises(fgl.FGLError) as e:
            fgl.fgl_noise_quantile(ref, lbar)
        assert e.value.code == fgl.FGL_EINVAL

def test_batch_size_bound_without_device_call(libpath):
    from paper_2603_13196_amd import fgl
    rc = fgl._lib.fgl_loglike_batch(None, None, 2**26 + 1, None, 0)
    assert rc == fgl.FGL_EINVAL    # a NULL model is refused first
    assert "NULL" in fgl.fgl_last_error()

def test_binding_fails_loudly_without_library(tmp_path, libpath):
    pkg = tmp_path / "pkgcopy"
    pkg.mkdir()
    shutil.copy(os.path.join(PKG, "fgl.py"), pkg / "fgl.py")
    (pkg / "__init__.py").write_text("")
    code = ("import sys; sys.path.insert(0, %r)\n"
            "try:\n    import pkgcopy.fgl\nexcept ImportError as e:\n"
            "    print('IMPORT-ERROR', e)\n" % str(tmp_path))
    p = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True)
    assert "IMPORT-ERROR" in p.stdout and "libfgl.so" in p.stdout


def test_product_path_never_uses_the_oracle():
    for dirpath, _, files in os.walk(PKG):
        for fn in files:
            if fn.endswith((".py", ".cpp", ".hip", ".h")):
                txt = open(os.path.join(dirpath, fn)).read()
                assert not re.search(r"\bimport\s+oracle|from\s+oracle|fgl_oracle|liboracle",
                                     txt), fn


def test_bench_refuses_more_than_one_gpu():
    """bench.py --gpus N with N > 1 exits with a message (one GPU only)."""
    import json
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    p = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert p.returncode == 2
    line = json.loads(p.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]
