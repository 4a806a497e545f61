"""The C-ABI library loads and exports every entry point that include/grnnd.h
declares; host-only calls (sizes, defaults, argument checks) behave as
documented. No GPU work is launched here."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "grnnd.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(grnnd_[a-z_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def g():
    import paper_2510_02774_amd as g
    if not os.path.exists(g.LIB_PATH):
        from paper_2510_02774_amd import build
        build.build()
    g.lib()
    return g


def test_every_declared_symbol_is_exported(g):
    names = _declared()
    assert len(names) >= 11
    L = C.CDLL(g.LIB_PATH)
    for n in names:
        assert hasattr(L, n), f"{n} declared in grnnd.h but not exported"
    for n in names:
        assert n in g.__all__, f"{n} has no binding of the same name"


def test_version_and_defaults(g):
    assert g.grnnd_version() >= 100
    p = g.grnnd_params_default(32, 4)
    assert (p.S, p.T1, p.T2, p.order, p.precision) == (32, 4, 4, 0, 0)
    assert abs(p.rho - 0.6) < 1e-7
    assert (p.reverse, p.check) == (g.REVERSE_HASH, 0)
    with pytest.raises(g.GrnndError):
        g.grnnd_params_default(0, 4)
    p.check = 2                                     # the pool check is 0 or 1
    with pytest.raises(g.GrnndError, match="check"):
        g.grnnd_workspace_size(1000, 128, 32, p)


def test_workspace_size_scales(g):
    a = g.grnnd_workspace_size(1000, 128, 32)
    b = g.grnnd_workspace_size(2000, 128, 32)
    assert 0 < a < b
    c = g.grnnd_workspace_size(1000, 130, 32)       # d % 4 != 0 adds a padded copy
    assert c >= a + 1000 * 132 * 4
    with pytest.raises(g.GrnndError):
        g.grnnd_workspace_size(1, 128, 32)
    with pytest.raises(g.GrnndError):
        g.grnnd_workspace_size(1000, 128, 65)


def test_argument_errors_before_any_launch(g):
    L = g.lib()
    ws = C.c_void_p(256)
    rc = L.grnnd_build(None, 100, 16, 0, 16, 2, 1, C.c_void_p(256), ws, 1 << 20, None)
    assert rc == -1 and "points" in g.grnnd_last_error()
    rc = L.grnnd_build(C.c_void_p(256), 100, 16, 0, 65, 2, 1, C.c_void_p(256), ws, 1 << 20, None)
    assert rc == -1
    rc = L.grnnd_build(C.c_void_p(256), 1, 16, 0, 16, 2, 1, C.c_void_p(256), ws, 1 << 20, None)
    assert rc == -1
    rc = L.grnnd_build(C.c_void_p(256), 100, 16, 7, 16, 2, 1, C.c_void_p(256), ws, 1 << 20, None)
    assert rc == -1 and "metric" in g.grnnd_last_error()
    rc = L.grnnd_build(C.c_void_p(256), 100, 16, 0, 16, 0, 1, C.c_void_p(256), ws, 1 << 20, None)
    assert rc == -1


def test_noalloc_refuses_sizes_beyond_its_scratch(g):
    """The allocation-free build checks its workspace need against the static
    scratch size before touching the device: too large is ENOSPACE."""
    L = g.lib()
    n = 1_000_000
    assert g.grnnd_workspace_size(n, 128, 32) > g.NOALLOC_SCRATCH_BYTES
    rc = L.grnnd_build_noalloc(C.c_void_p(256), n, 128, 0, 32, None, 1, C.c_void_p(256), None,
                               None, None)
    assert rc == -2 and "scratch" in g.grnnd_last_error()
    rc = L.grnnd_build_noalloc(C.c_void_p(256), 1, 128, 0, 32, None, 1, C.c_void_p(256), None,
                               None, None)
    assert rc == -1


def test_medoid_and_search_argument_errors(g):
    L = g.lib()
    rc = L.grnnd_medoid(None, 10, 4, C.c_void_p(256), C.c_void_p(256), 1 << 20, None)
    assert rc == -1 and "null" in g.grnnd_last_error()
    rc = L.grnnd_medoid(C.c_void_p(256), 0, 4, C.c_void_p(256), C.c_void_p(256), 1 << 20, None)
    assert rc == -1
    need = g.grnnd_search_workspace_size(1000, 16, 0)
    rc = L.grnnd_medoid(C.c_void_p(256), 1000, 16, C.c_void_p(256), C.c_void_p(256), 64, None)
    assert rc == -2 and need > 64
    # the search's workspace grows with the medoid's scratch (FP64 distances)
    assert g.grnnd_search_workspace_size(100000, 16, 10) > 100000 * 8
    rc = L.grnnd_search(C.c_void_p(256), 100, 16, 0, C.c_void_p(256), 16, 100, C.c_void_p(256),
                        1, 10, 16, C.c_void_p(256), C.c_void_p(256), C.c_void_p(256), 1 << 20,
                        None)
    assert rc == -1 and "entry" in g.grnnd_last_error()


def test_batch_argument_errors(g):
    L = g.lib()
    with pytest.raises(g.GrnndError):
        g.grnnd_batch_workspace_size([100, 1], 16, 16)      # a collection below 2 points
    with pytest.raises(g.GrnndError):
        g.grnnd_batch_workspace_size([100] * 65, 16, 16)    # more than 64 collections
    one = g.grnnd_workspace_size(300, 16, 16)
    two = g.grnnd_batch_workspace_size([100, 200], 16, 16)
    assert two > one                                       # plus the concatenated points
    rc = L.grnnd_build_batch(None, 2, 16, 0, 16, None, None, C.c_void_p(256), 1 << 20, None)
    assert rc == -1
