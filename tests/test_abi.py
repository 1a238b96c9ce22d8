"""The C-ABI library loads and exports every function include/hbspeel.h
declares; host-side argument validation answers without touching a GPU."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hbspeel.h")
LIB = os.path.join(ROOT, "paper_1503_07152_amd", "libhbspeel.so")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?(?:int|void|char)\s*\*?\s*(\w+)\s*\(", txt, flags=re.M)
    return sorted(set(names))


def test_header_lists_the_boundary():
    names = declared_functions()
    for must in ("hodlr_compress", "hbs_compress", "hss_apply", "hss_apply_adjoint",
                 "hss_apply_backward", "hbs_compress_batched", "hm_gauss", "hm_operator_apply",
                 "hm_hbs_info", "hm_hbs_generators", "hm_set_allocator", "hm_hbs_free",
                 "hm_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "build first: python -c 'import __graft_entry__ as g; g.build()'"
    lib = C.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_names_match_boundary():
    import paper_1503_07152_amd as hm
    for n in ("hbs_compress", "hodlr_compress", "hss_apply", "hss_apply_adjoint",
              "hss_apply_backward", "hbs_compress_batched", "hm_gauss", "hm_operator_apply"):
        assert callable(getattr(hm, n))


@pytest.mark.parametrize("kw,code", [
    (dict(n=0, leaf_size=64, rank=10, oversample=10), -1),
    (dict(n=1024, leaf_size=0, rank=10, oversample=10), -1),
    (dict(n=1024, leaf_size=64, rank=0, oversample=10), -1),
    (dict(n=1024, leaf_size=64, rank=10, oversample=-1), -1),
    (dict(n=1024, leaf_size=64, rank=10, oversample=10, tol=1.5), -1),
    (dict(n=1024, leaf_size=64, rank=40, oversample=10), -6),   # r > HM_MAX_SAMPLES
])
def test_invalid_options_rejected_on_host(kw, code):
    import paper_1503_07152_amd as hm
    opts = hm.Options(**kw)
    op = hm._Operator()
    op.kind = hm.HM_OP_KERNEL
    op.points = 1   # never dereferenced: options fail first
    h = C.c_void_p(123)
    rc = hm.lib.hbs_compress(C.byref(opts.c), C.byref(op), None, C.byref(h))
    assert rc == code
    assert h.value is None               # out set to NULL on error
    assert hm.lib.hm_last_error().decode() != ""


def test_invalid_operator_rejected_on_host():
    import paper_1503_07152_amd as hm
    opts = hm.Options(1024, 64, 10, 10)
    op = hm._Operator()
    op.kind = 99
    h = C.c_void_p()
    assert hm.lib.hbs_compress(C.byref(opts.c), C.byref(op), None, C.byref(h)) == -1
    op.kind = hm.HM_OP_DENSE          # dense without a matrix
    assert hm.lib.hbs_compress(C.byref(opts.c), C.byref(op), None, C.byref(h)) == -1


def test_allocator_and_views_argument_checks_on_host():
    import paper_1503_07152_amd as hm
    # exactly one of alloc / free set is an argument error; both NULL restores hipMalloc
    alloc = hm.ALLOC_FN(lambda ctx, n, s: None)
    assert hm.lib.hm_set_allocator(alloc, hm.FREE_FN(), None) == -1
    assert hm.lib.hm_set_allocator(hm.ALLOC_FN(), hm.FREE_FN(lambda c, p, s: None), None) == -1
    assert hm.lib.hm_set_allocator(hm.ALLOC_FN(), hm.FREE_FN(), None) == 0
    v = hm._Views()
    assert hm.lib.hm_hbs_generators(None, C.byref(v)) == -1
    assert "generators" in hm.lib.hm_last_error().decode()


@pytest.mark.parametrize("height,width,ch,cv,code", [
    (0, 41, 1, 1, -1),        # no rows
    (8, 40, 1, 1, -1),        # even width: no middle column
    (8, 1, 1, 1, -1),         # no sides
    (8, 67, 1, 1, -6),        # sides wider than 32 columns
    (8, 41, None, 1, -1),     # no conductivities
    (8, 41, 1, None, -1),     # vertical bars missing with more than one row
])
def test_frontal_arguments_rejected_on_host(height, width, ch, cv, code):
    import paper_1503_07152_amd as hm
    f = C.c_void_p(123)
    rc = hm.lib.hm_frontal_create(height, width, ch, cv, None, C.byref(f))
    assert rc == code
    assert f.value is None
    assert hm.lib.hm_frontal_apply(None, 1, 1, 8, 1, 8, None) == -1
