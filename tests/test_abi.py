"""The C-ABI library: it loads, exports every symbol ``include/aa.h`` declares,
and rejects bad arguments on the host before touching a device (no GPU needed:
argument checks come first and nothing is enqueued)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "aa.h")


@pytest.fixture(scope="module")
def L():
    from paper_2110_09667_amd import aa
    if not os.path.exists(aa.LIB_PATH):
        pytest.skip("libaa.so not built")
    return aa.lib()


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(aa_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_binding_symbols():
    from paper_2110_09667_amd import aa
    assert set(declared_symbols()) == set(aa.SYMBOLS)


def test_every_declared_symbol_is_exported(L):
    for name in declared_symbols():
        assert hasattr(L, name), name


def test_version(L):
    from paper_2110_09667_amd import aa
    assert "gfx950" in aa.aa_version()


def test_workspace_size_and_argument_errors(L):
    from paper_2110_09667_amd import aa
    b = C.c_size_t(0)
    assert L.aa_workspace_size(4096, 5, aa.MGS, 0, C.byref(b)) == 0
    full = b.value
    # Q, Delta g ring, f_prev, g_prev, W: (2m + 3) vectors of ldq >= n doubles
    assert full >= (2 * 5 + 3) * 4096 * 8
    assert L.aa_workspace_size(4096, 5, aa.MGS, aa.QR_ONLY, C.byref(b)) == 0
    assert b.value < full
    assert L.aa_workspace_size(0, 5, aa.MGS, 0, C.byref(b)) == -1
    assert L.aa_workspace_size(10, 0, aa.MGS, 0, C.byref(b)) == -1
    assert L.aa_workspace_size(10, 66, aa.MGS, 0, C.byref(b)) == -1
    assert L.aa_workspace_size(10, 65, aa.ICWY, 0, C.byref(b)) == -1
    assert L.aa_workspace_size(10, 65, aa.ICWY, aa.QR_ONLY, C.byref(b)) == -1
    # a 65th column only for the QR update on its own: the LSP solve and
    # aa_step reach 64 columns
    for v in (aa.MGS, aa.CGS2, aa.DCGS2):
        assert L.aa_workspace_size(10, 65, v, 0, C.byref(b)) == -1
        assert L.aa_workspace_size(10, 65, v, aa.QR_ONLY, C.byref(b)) == 0
        assert L.aa_workspace_size(10, 64, v, 0, C.byref(b)) == 0
    assert L.aa_workspace_size(10, 5, 7, 0, C.byref(b)) == -1
    assert L.aa_workspace_size(10, 5, aa.MGS, 0, None) == -1
    ctx = C.c_void_p()
    # null / misaligned workspace and short workspace are refused up front
    assert L.aa_init(C.byref(ctx), 100, 4, aa.MGS, 0, None, 1 << 20, None) == -1
    assert L.aa_init(C.byref(ctx), 100, 4, aa.MGS, 0, 8, 1 << 20, None) == -1
    assert L.aa_init(C.byref(ctx), 100, 4, aa.MGS, 0, 4096, 16, None) == -5
    assert L.aa_init(None, 100, 4, aa.MGS, 0, 4096, 1 << 20, None) == -1
    # null contexts
    assert L.aa_step(None, None, None, None) == -1
    assert L.aa_qr_add(None, None) == -1
    assert L.aa_qr_delete(None) == -1
    assert L.aa_problem_apply(4, 8, 0.1, 1.0, 0.0, 8, 16, 24, None) == -1
    assert L.aa_problem_apply(1, 8, 0.1, 1.0, 0.0, 8, 16, 16, None) == -1
