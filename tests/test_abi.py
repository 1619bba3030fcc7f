"""The C-ABI library loads and exports every symbol include/pkd.h declares;
host-side argument checks work without a GPU (no compute calls here)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pkd.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pkd_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    import paper_2411_09275_amd as pk
    if not os.path.exists(pk.LIB_PATH):
        pytest.skip("libpkd.so not built")
    return pk.lib()


def test_header_matches_binding_list():
    import paper_2411_09275_amd as pk
    assert _declared() == sorted(pk.EXPORTS)


def test_every_declared_symbol_is_exported(L):
    for name in _declared():
        assert hasattr(L, name), name


def test_defaults_and_strerror(L):
    import paper_2411_09275_amd as pk
    p = pk._Params()
    L.pkd_default_params(C.byref(p), 3)
    assert (p.dim, p.lambda_, p.leaf_size, p.oversample, p.alpha_num, p.alpha_den, p.seed) == (3, 6, 32, 32, 3, 10, 42)
    t = pk._Tuning()
    L.pkd_default_tuning(C.byref(t))
    assert t.tile_points == 2048
    for code in range(0, -8, -1):
        assert L.pkd_strerror(code)


def test_parameter_validation_before_any_device_work(L):
    import paper_2411_09275_amd as pk
    out = C.c_void_p()
    bad = [dict(dim=0), dict(dim=10), dict(lambda_=0), dict(lambda_=9), dict(leaf_size=0), dict(oversample=0),
           dict(alpha_num=5, alpha_den=10), dict(alpha_den=0), dict(oversample=65),
           dict(oversample=33), dict(lambda_=7, oversample=32), dict(lambda_=8, oversample=16),
           dict(dim=7, leaf_size=1)]
    # a sample above 2048 points is unsupported, and so is a 7-D sample of 2048
    # with leaves of one point (its finisher workgroup would need over 160 KB of LDS)
    expect = [-3, -3, -1, -1, -1, -1, -1, -1, -3, -3, -3, -3, -3]
    for change, code in zip(bad, expect):
        p = pk._Params()
        L.pkd_default_params(C.byref(p), 7 if change.get("dim") == 7 else 2)
        for k, v in change.items():
            setattr(p, k, v)
        assert L.pkd_build(C.byref(p), None, None, None, None, 10, C.byref(out)) == code, change
    p = pk._Params()
    L.pkd_default_params(C.byref(p), 2)
    assert L.pkd_build(C.byref(p), None, None, None, None, -1, C.byref(out)) == -1
    assert L.pkd_build(C.byref(p), None, None, None, None, 5, C.byref(out)) == -1     # null inputs
    t = pk._Tuning()
    L.pkd_default_tuning(C.byref(t))
    t.tile_points = 3000
    assert L.pkd_build(C.byref(p), C.byref(t), None, None, None, 0, C.byref(out)) == -1
    L.pkd_default_tuning(C.byref(t))
    assert t.cand_shift_bias == 0
    for bias in (-5, 5, 100):
        t.cand_shift_bias = bias
        assert L.pkd_build(C.byref(p), C.byref(t), None, None, None, 0, C.byref(out)) == -1
    L.pkd_default_tuning(C.byref(t))
    assert t.update_events == 0
    for events in (-1, 3):
        t.update_events = events
        assert L.pkd_build(C.byref(p), C.byref(t), None, None, None, 0, C.byref(out)) == -1
    assert L.pkd_knn(None, None, None, 1, 1, None, None) == -1
    assert L.pkd_range_count(None, None, None, None, 1, None) == -1
    assert L.pkd_size(None, None) == -1
