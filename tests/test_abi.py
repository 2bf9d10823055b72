"""The C ABI library builds, loads and exports every function include/felog.h
declares; the oracle stays independent of the HIP path.  CPU only."""
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "felog.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(felog_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2606_22180_amd import build, felog
    if not os.path.exists(build.LIB):
        build.build()
    return felog.load()


def test_header_declares_functions():
    names = _declared()
    assert "felog_walks_generate" in names and "felog_train_epoch" in names
    assert "felog_feedback" in names and "felog_run" in names


def test_library_exports_every_declared_symbol(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", lib._name], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\b(felog_[a-z0-9_]+)\b", out))
    missing = [n for n in _declared() if n not in exported]
    assert not missing, missing


def test_binding_covers_every_declared_symbol(lib):
    from paper_2606_22180_amd import felog
    assert sorted(felog.SIGNATURES) == _declared()


def test_errors_without_a_device_are_reported(lib):
    import ctypes
    if os.path.exists("/dev/kfd"):
        pytest.skip("a GPU is present; covered by the GPU tests")
    h = ctypes.c_void_p()
    st = lib.felog_ctx_create(0, None, 0, ctypes.byref(h))
    assert st != 0 and h.value is None
    assert lib.felog_last_error()
    # NULL handles are rejected, destroy(NULL) is a no-op
    assert lib.felog_ctx_create(0, None, 0, None) == -1
    lib.felog_graph_destroy(None)
    lib.felog_walks_destroy(None)
    lib.felog_model_destroy(None)
    lib.felog_active_destroy(None)
    lib.felog_ctx_destroy(None)


def test_oracle_is_independent_of_the_hip_path():
    """The oracle neither includes nor imports the HIP library, and the HIP
    sources never mention the oracle."""
    odir = os.path.join(ROOT, "oracle")
    for f in os.listdir(odir):
        if f.endswith((".c", ".h", ".py")):
            text = open(os.path.join(odir, f)).read()
            assert "paper_2606_22180_amd" not in text.replace(
                "(``paper_2606_22180_amd``)", "")
            assert "csrc" not in text and "felog.h" not in text
    cdir = os.path.join(ROOT, "paper_2606_22180_amd")
    for dirpath, _, files in os.walk(cdir):
        for f in files:
            if f.endswith((".hip", ".cpp", ".h", ".py")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text
                assert "felog_oracle" not in text


def test_no_cuda_or_triton_sources():
    for dirpath, _, files in os.walk(ROOT):
        if "/." in dirpath or "_work" in dirpath:
            continue
        for f in files:
            assert not f.endswith((".cu", ".cuh")), f
            if f.endswith(".py") and "test_abi" not in f:
                assert "import triton" not in open(os.path.join(dirpath, f)).read()


def test_product_import_does_not_pull_the_oracle():
    code = ("import sys; sys.path.insert(0, %r); import paper_2606_22180_amd.felog as f; "
            "f.load(); assert 'oracle' not in sys.modules" % ROOT)
    subprocess.run([sys.executable, "-c", code], check=True)
