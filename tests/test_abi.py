"""CPU checks of the C ABI: the built library loads and exports every
function include/cbs.h declares, and the binding declares each of them."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cbs.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cbs_[a-z_]+)\s*\(", src)))


def test_header_declares_the_lifecycle():
    names = _declared()
    for fn in ("cbs_create_from_ldu", "cbs_update_values", "cbs_setup", "cbs_solve",
               "cbs_solve_transpose", "cbs_destroy", "cbs_create_batch_from_ldu", "cbs_gradient"):
        assert fn in names


def test_library_exports_every_declared_symbol():
    import paper_2403_07882_amd as P
    L = P.lib()
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing
    bound = {name for name, _, _ in P.binding.SIGNATURES}
    assert set(_declared()) == bound


def test_error_strings_without_gpu():
    import paper_2403_07882_amd as P
    L = P.lib()
    assert L.cbs_error_string(-3) == b"CBS_ERR_SINGULAR"
    assert L.cbs_error_string(1) == b"CBS_NOT_CONVERGED"
    o = P.default_options()
    assert o.tol == 1e-8 and o.restart == 30 and o.precond == P.PREC_AMG


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    import paper_2403_07882_amd.binding as B
    monkeypatch.setattr(B, "_lib", None)
    monkeypatch.setattr(B, "LIB_PATH", str(tmp_path / "nope.so"))
    with pytest.raises(ImportError):
        B.lib()


def test_options_and_stats_layout_match_the_header():
    """The ctypes structures list the header's fields in the header's order."""
    import paper_2403_07882_amd as P
    src = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    for cname, cls in (("cbs_options", P.Options), ("cbs_stats", P.Stats)):
        body = re.search(r"typedef struct %s \{(.*?)\} %s;" % (cname, cname), src, re.S).group(1)
        fields = re.findall(r"\b(int32_t|double)\s+([a-z_0-9]+)\s*;", body)
        assert [f for _, f in fields] == [f for f, _ in cls._fields_], cname
        kinds = {"int32_t": "c_int", "double": "c_double"}
        for (ct, _), (_, pt) in zip(fields, cls._fields_):
            assert pt.__name__.startswith(kinds[ct]), (cname, ct, pt)


def test_argument_errors_without_gpu():
    """Every entry point rejects a NULL handle or bad sizes with CBS_ERR_ARG
    before touching the device; cbs_destroy(NULL) is allowed."""
    import ctypes as C
    import paper_2403_07882_amd as P
    L = P.lib()
    o, st = P.default_options(), P.Stats()
    calls = [
        lambda: L.cbs_setup(None, C.byref(o)),
        lambda: L.cbs_solve(None, None, None, C.byref(st)),
        lambda: L.cbs_solve_transpose(None, None, None, C.byref(st)),
        lambda: L.cbs_solve_batch(None, None, None, C.byref(st)),
        lambda: L.cbs_get_mirror(None, None),
        lambda: L.cbs_set_allocator(None, None),
        lambda: L.cbs_apply_precond(None, None, None),
        lambda: L.cbs_apply_precond_transpose(None, None, None),
        lambda: L.cbs_spmv(None, None, None, 0),
        lambda: L.cbs_level_apply(None, 0, 0, None, None, None, None),
        lambda: L.cbs_gradient(None, None, None, None, None, None),
        lambda: L.cbs_update_values(None, None, None, None),
        lambda: L.cbs_assemble_luo(None, None, None, None, None, 1.4),
        lambda: L.cbs_assemble_pu(None, None, None, None, None, None, None, None, None),
    ]
    for call in calls:
        assert call() == P.ERR_ARG
    assert L.cbs_destroy(None) == 0
    h = C.c_void_p()
    assert L.cbs_create_from_ldu(C.byref(h), 10, 0, 7, None, None, None, None, None, None) == P.ERR_ARG
    assert b"bdim" in L.cbs_last_error()
    assert not h.value
