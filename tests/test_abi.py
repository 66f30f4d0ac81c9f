"""The C ABI without a GPU: the library loads, exports every entry point the
header declares, and rejects invalid arguments with SVCONV_EINVAL (or
SVCONV_EUNSUPPORTED) before making any HIP call."""

import ctypes
import os
import re

import pytest

from paper_1209_5823_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "svconv.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(svconv_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    return _lib.load()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 19
    for n in names:
        assert hasattr(lib, n), n
    # and the binding knows every one of them
    assert set(names) == set(_lib.SIGNATURES)


def _create(lib, H=64, W=64, h=3, sig=(1.5,), deg=(2,), ds=2, prec=0):
    p = ctypes.c_void_p()
    s = (ctypes.c_double * len(sig))(*sig)
    d = (ctypes.c_int * len(deg))(*deg)
    rc = lib.svconv_plan_create(ctypes.byref(p), H, W, h, len(sig), s, d, ds, prec)
    return rc, p


@pytest.mark.parametrize("kw,status", [
    (dict(H=0), _lib.EINVAL),
    (dict(W=-3), _lib.EINVAL),
    (dict(h=-1), _lib.EINVAL),
    (dict(sig=(-1.0,)), _lib.EINVAL),
    (dict(sig=(float("nan"),)), _lib.EINVAL),
    (dict(sig=(0.0,), deg=(1,)), _lib.EINVAL),      # delta basis must have degree 0
    (dict(deg=(-2,)), _lib.EINVAL),
    (dict(ds=-1), _lib.EINVAL),
    (dict(prec=9), _lib.EINVAL),
    (dict(h=32), _lib.EUNSUPPORTED),
    (dict(ds=7), _lib.EUNSUPPORTED),
    (dict(deg=(10,)), _lib.EUNSUPPORTED),           # 66 bases > 64
    (dict(sig=(1.0, 2.0), deg=(6, 6), ds=6), _lib.EUNSUPPORTED),  # N*M = 56*28 > 1024
])
def test_plan_create_rejects_before_any_device_call(lib, kw, status):
    rc, p = _create(lib, **kw)
    assert rc == status
    assert not p.value
    assert lib.svconv_last_error().decode() != ""


def test_null_plan_and_null_pointers(lib):
    E = _lib.EINVAL
    assert lib.svconv_plan_create(None, 8, 8, 1, 1, None, None, 0, 0) == E
    assert lib.svconv_plan_create_dfb(None, 8, 8, 1, 0, 0) == E
    assert lib.svconv_plan_set_frame(None, 0, 0, 8, 8) == E
    assert lib.svconv_plan_set_stream(None, None) == E
    assert lib.svconv_plan_set_precision(None, 0) == E
    assert lib.svconv_plan_set_form(None, 0) == E
    assert lib.svconv_plan_set_pedestal(None, 1.0) == E
    assert lib.svconv_plan_sizes(None, None, None) == E
    assert lib.svconv_plan_get_basis(None, None) == E
    assert lib.svconv_forward(None, None, None, None) == E
    assert lib.svconv_difference(None, None, None, None, None) == E
    assert lib.svconv_backward(None, None, None, None, None, None) == E
    assert lib.svconv_loss_grad(None, None, None, None, None) == E
    assert lib.svconv_normal_matrix(None, None, None, None) == E
    assert lib.svconv_cholesky_factor(None, None, 4) == E
    assert lib.svconv_cholesky_solve(None, None, None, None, 4) == E
    assert lib.svconv_gn_step(None, None, None, None, None, None, None, None, None) == E
    assert lib.svconv_normal_equations(None, None, None, None, None, None) == E
    assert lib.svconv_ls_step(None, None, None, None, None, None, None, None, None, None, None) == E
    assert lib.svconv_plan_destroy(None) == _lib.OK


@pytest.mark.parametrize("args,status", [
    ((0, 8, 1, 0, 0), _lib.EINVAL),
    ((8, 8, -1, 0, 0), _lib.EINVAL),
    ((8, 8, 1, -1, 0), _lib.EINVAL),
    ((8, 8, 1, 0, 7), _lib.EINVAL),
    ((8, 8, 32, 0, 0), _lib.EUNSUPPORTED),
    ((8, 8, 7, 2, 0), _lib.EUNSUPPORTED),      # 225 delta bases x 6 terms > 1024
])
def test_dfb_plan_rejects_before_any_device_call(lib, args, status):
    p = ctypes.c_void_p()
    assert lib.svconv_plan_create_dfb(ctypes.byref(p), *args) == status
    assert not p.value


def test_strerror(lib):
    for st in (0, -1, -2, -3, -4, -5):
        assert lib.svconv_strerror(st).decode()
    assert lib.svconv_strerror(-99).decode() == "unknown status"


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        _lib.load()


def test_pipeline_rejects_before_any_device_call(lib):
    E = _lib.EINVAL
    q = ctypes.c_void_p()
    assert lib.svconv_pipeline_create(None, 2, ctypes.byref(q)) == E
    assert not q.value
    assert lib.svconv_pipeline_create(None, 2, None) == E
    assert lib.svconv_pipeline_run(None, 1, None, None, None, None) == E
    assert lib.svconv_pipeline_destroy(None) == _lib.OK
    assert lib.svconv_host_alloc(16, None) == E
    p = ctypes.c_void_p()
    assert lib.svconv_host_alloc(0, ctypes.byref(p)) == E
    assert not p.value
    assert lib.svconv_host_free(None) == _lib.OK


def test_ois_entry_points_reject_before_any_device_call(lib):
    E = _lib.EINVAL
    n = ctypes.c_int()
    assert lib.svconv_stamp_mask(None, None, 0.0, 1.0, 0.1, 3, 0, 2, None, ctypes.byref(n)) == E
    assert lib.svconv_plan_set_background(None, 1) == E
    assert lib.svconv_add_background(None, None, None) == E
    assert lib.svconv_pcg_fit(None, None, None, None, None, 1, None, None, None, None) == E


@pytest.mark.parametrize("kw,status", [
    (dict(h=13), _lib.EUNSUPPORTED),
    (dict(h=0), _lib.EUNSUPPORTED),
    (dict(d_s=3), _lib.EUNSUPPORTED),
    (dict(precision=0), _lib.EUNSUPPORTED),
    (dict(degrees=(9, 9, 9, 9)), _lib.EUNSUPPORTED),     # 220 bases, 40 row factors
    (dict(degrees=(6, 6, 6, 6, 6)), _lib.EUNSUPPORTED),  # 35 row factors > 32
    (dict(sigmas=(0.0,), degrees=(0,)), _lib.EUNSUPPORTED),
    (dict(H=0), _lib.EINVAL),
    (dict(precision=9), _lib.EINVAL),
    (dict(sigmas=(-1.0,), degrees=(1,)), _lib.EINVAL),
])
def test_noalloc_rejects_before_any_device_call(lib, kw, status):
    H, W = kw.get("H", 16), 16
    deg = kw.get("degrees", (1,))
    sig = kw.get("sigmas", (1.5,) * len(deg))
    s = (ctypes.c_double * len(sig))(*sig)
    d = (ctypes.c_int * len(deg))(*deg)
    dummy = ctypes.c_void_p(16)   # never dereferenced: validation fails first
    rc = lib.svconv_difference_noalloc(H, W, kw.get("h", 3), len(sig), s, d, kw.get("d_s", 2),
                                       kw.get("precision", 5), 0.0, dummy, dummy, dummy,
                                       ctypes.c_void_p(32), None)
    assert rc == status
    assert lib.svconv_last_error().decode() != ""


def test_build_reports_no_register_spills():
    # build() records the compiler's resource-usage report of every kernel and
    # fails on a spill; the report of the library in this tree must show none
    import json
    path = os.path.join(ROOT, "_build", "resource_usage.json")
    if not os.path.exists(path):
        pytest.skip("no resource-usage report: the library was not built in this tree")
    with open(path) as f:
        usage = json.load(f)
    assert len(usage) > 100
    spills = {k: v["scratch"] for k, v in usage.items() if v.get("scratch", 0)}
    assert not spills, spills
