"""C-ABI library checks that need no GPU: it loads, exports every symbol the
header declares, reports missing devices cleanly, and the Python binding
declares the same surface."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gpbo.h")
LIB = os.path.join(ROOT, "paper_2403_08131_amd", "libgpbo.so")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(gpbo_[a-z_]+)\s*\(", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2403_08131_amd import build
        build.build()
    return C.CDLL(LIB)


def test_header_declares_the_documented_surface():
    names = _declared()
    for must in ["gpbo_ctx_create", "gpbo_fit", "gpbo_fit_batched", "gpbo_score",
                 "gpbo_score_batched", "gpbo_mlp_train", "gpbo_mlp_prescreen", "gpbo_topk"]:
        assert must in names
    assert len(names) >= 24


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    from paper_2403_08131_amd import gpbo
    assert sorted(gpbo._SIGS) == _declared()


def test_status_strings_and_version(lib):
    lib.gpbo_status_string.restype = C.c_char_p
    assert lib.gpbo_status_string(0) == b"ok"
    assert b"positive definite" in lib.gpbo_status_string(2)
    assert lib.gpbo_status_string(99) == b"unknown status"
    assert lib.gpbo_version() >= 10000
    lib.gpbo_mlp_nparams.restype = C.c_int64
    assert lib.gpbo_mlp_nparams(20, 256) == 71425


def test_ctx_create_without_device_fails_cleanly(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = C.c_void_p()
    st = lib.gpbo_ctx_create(0, None, None, C.byref(h))
    assert st == 5  # GPBO_E_HIP
    assert not h.value
    lib.gpbo_last_error.restype = C.c_char_p
    assert b"device" in lib.gpbo_last_error(None)


def test_null_handles_are_rejected(lib):
    assert lib.gpbo_fit(None, None, None, None, None) == 1
    assert lib.gpbo_score(None, None, 0, None, 1, None, None, None, None, None) == 1
    assert lib.gpbo_ctx_destroy(None) == 0
    assert lib.gpbo_model_free(None) == 0


def test_library_starts_no_process():
    """The library runs inside processes that drive the GPU: no shell, fork or
    exec of another program from its sources."""
    csrc = os.path.join(ROOT, "paper_2403_08131_amd", "csrc")
    bad = re.compile(r"\b(system|popen|fork|vfork|execv|execvp|execl|execlp|posix_spawn)\s*\(")
    hits = []
    for name in sorted(os.listdir(csrc)):
        text = open(os.path.join(csrc, name)).read()
        text = re.sub(r"//[^\n]*", "", text)
        hits += [(name, m.group(0)) for m in bad.finditer(text)]
    assert not hits, hits
