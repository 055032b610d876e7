"""The C ABI library loads, exports every declared entry point, and rejects
bad arguments on the host before touching a GPU."""
import ctypes
import os
import re

import pytest

from paper_2310_15235_amd import api

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "trevr2.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(trevr_[A-Za-z_]+)\s*\(", src)))


def test_header_and_binding_agree():
    assert _declared() == sorted(api.EXPORTED)


def test_library_exports_every_symbol():
    L = api.lib()
    for name in _declared():
        assert hasattr(L, name), name


def test_status_strings():
    L = api.lib()
    for s in range(6):
        assert len(L.trevr_status_string(s)) > 0


@pytest.mark.parametrize("kw", [dict(nside=3), dict(nside=0), dict(nside=32), dict(leaf_size=0),
                                dict(n_bands=0), dict(n_bands=17), dict(theta=-1.0),
                                dict(theta=float("nan")), dict(rpp_min=-1.0), dict(flags=128),
                                dict(flags=32, target=(float("nan"), 0.0, 0.0))])
def test_invalid_params_rejected(kw):
    p = api.make_params(**kw)
    with pytest.raises(api.TrevrError) as e:
        api.workspace_bytes(p, 100)
    assert e.value.status == api.E_INVALID


def test_invalid_sizes_and_pointers():
    p = api.make_params()
    for n in (0, -5, 2 ** 31):
        with pytest.raises(api.TrevrError):
            api.workspace_bytes(p, n)
    tb, sb = api.workspace_bytes(p, 1000)
    assert tb > 0 and sb > 0
    h = ctypes.c_void_p()
    st = api.lib().trevr_build_tree(ctypes.byref(p), 1000, None, None, None, None, None, None,
                                    None, None, 0, None, ctypes.byref(h))
    assert st == api.E_INVALID and not h.value


def test_workspace_grows_with_n_and_bands():
    a, _ = api.workspace_bytes(api.make_params(n_bands=1), 1000)
    b, _ = api.workspace_bytes(api.make_params(n_bands=3), 1000)
    c, _ = api.workspace_bytes(api.make_params(n_bands=1), 4000)
    assert b > a and c > a


def test_unknown_handle_rejected():
    L = api.lib()
    bogus = ctypes.c_void_p(12345678)
    assert L.trevr_check(bogus) == api.E_STATE
    assert L.trevr_tree_destroy(bogus) == api.E_STATE
    c = api.Counters()
    assert L.trevr_get_counters(bogus, ctypes.byref(c)) == api.E_STATE


def _struct_fields(name):
    import re
    text = open(os.path.join(ROOT, "include", "trevr2.h")).read()
    body = re.search(r"typedef struct %s \{(.*?)\} %s;" % (name, name), text, re.S).group(1)
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    fields = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        m = re.match(r"(\w+)\s+(\w+)(\[\d+\])?$", decl)
        assert m, decl
        fields.append(m.group(2))
    return fields


def test_binding_structs_match_header():
    """The ctypes mirrors of the C structs list the header's fields in order."""
    assert [f for f, _ in api.Counters._fields_] == _struct_fields("trevr_counters")
    assert [f for f, _ in api.Params._fields_] == _struct_fields("trevr_params")


def test_tune_rejects_unknown_handle():
    L = api.lib()
    bogus = ctypes.c_void_p(0x1234)
    assert L.trevr_tree_tune(bogus, api.TUNE_STACK, 256) == api.E_STATE


def test_forest_arguments_checked_on_host():
    L = api.lib()
    P = (api.Params * 2)(api.make_params(), api.make_params(n_bands=2))
    sz = ctypes.c_size_t()
    ok = (ctypes.c_int64 * 3)(0, 100, 250)
    assert L.trevr_forest_workspace_bytes(P, 2, ctypes.cast(ok, ctypes.c_void_p),
                                          ctypes.byref(sz)) == api.OK
    one, _ = api.workspace_bytes(api.make_params(), 100)
    two, _ = api.workspace_bytes(api.make_params(n_bands=2), 150)
    assert sz.value >= one + two
    for bad, S in (((0, 100, 100), 2), ((5, 100, 250), 2), ((0, 100, 250), 0)):
        arr = (ctypes.c_int64 * 3)(*bad)
        assert L.trevr_forest_workspace_bytes(P, S, ctypes.cast(arr, ctypes.c_void_p),
                                              ctypes.byref(sz)) == api.E_INVALID
    h = ctypes.c_void_p()
    st = L.trevr_build_forest(P, 2, ctypes.cast(ok, ctypes.c_void_p), *([None] * 8), 0, None,
                              ctypes.byref(h))
    assert st == api.E_INVALID and not h.value


def test_unknown_forest_handle_rejected():
    L = api.lib()
    bogus = ctypes.c_void_p(87654321)
    sz = ctypes.c_size_t()
    assert L.trevr_forest_check(bogus) == api.E_STATE
    assert L.trevr_forest_destroy(bogus) == api.E_STATE
    assert L.trevr_forest_plan_bytes(bogus, ctypes.byref(sz)) == api.E_STATE
    assert L.trevr_forest_job_log(bogus, 1 << 20) == api.E_STATE
    assert L.trevr_compute_J_batched(bogus, None, None, None, None, 0, None) == api.E_STATE
