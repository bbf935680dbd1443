"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/kgs.h declares, and rejects invalid arguments with the
documented status before it touches the device."""
import ctypes
import os
import re

import pytest

from paper_2502_09537_amd import kgs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(kgs.LIB_PATH):
        from paper_2502_09537_amd import build

        build.build()
    return kgs.lib()


def declared_functions():
    names = set()
    for f in os.listdir(os.path.join(ROOT, "include")):
        if f.endswith(".h"):
            text = open(os.path.join(ROOT, "include", f)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(kgs_[a-z_0-9]+)\s*\(", text))
    return names


def test_library_exports_every_declared_function(L):
    names = declared_functions()
    assert names, "no declarations found"
    for name in sorted(names):
        assert hasattr(L, name), f"{name} declared in include/ but not exported"
    assert names == set(kgs.EXPORTS), "binding and header disagree"


def test_status_strings(L):
    for code, name in enumerate(["KGS_OK", "KGS_EINVAL", "KGS_EODDN", "KGS_ESINGULAR",
                                 "KGS_ENOMEM", "KGS_EDEVICE", "KGS_ENONFINITE"]):
        assert kgs.status_string(code) == name
    assert kgs.status_string(99) == "KGS_UNKNOWN"


def _init_status(cfg, ptr=1):
    h = ctypes.c_void_p()
    rc = kgs.lib().kgs_init(ctypes.byref(cfg) if cfg is not None else None, ptr, ptr, ptr, ptr,
                            kgs.KGS_HOST, None, ctypes.byref(h))
    assert h.value is None
    return rc


def good(**kw):
    base = dict(dim=2, n=8, lo=-1.0, hi=1.0, tau=0.01)
    base.update(kw)
    return kgs.make_config(**base)


@pytest.mark.parametrize("cfg,status", [
    (dict(dim=0), kgs.KGS_EINVAL),
    (dict(dim=4), kgs.KGS_EINVAL),
    (dict(n=0), kgs.KGS_EINVAL),
    (dict(n=7), kgs.KGS_EODDN),
    (dict(hi=-1.0), kgs.KGS_EINVAL),
    (dict(hi=float("inf")), kgs.KGS_EINVAL),
    (dict(tau=0.0), kgs.KGS_EINVAL),
    (dict(tau=float("nan")), kgs.KGS_EINVAL),
    (dict(kappa1=float("nan")), kgs.KGS_EINVAL),
    (dict(gamma=float("inf")), kgs.KGS_EINVAL),
    (dict(precision=2), kgs.KGS_EINVAL),
])
def test_invalid_config_rejected_before_device_use(L, cfg, status):
    assert _init_status(good(**cfg)) == status
    assert kgs.last_error(None) != ""
    assert kgs.required_bytes(good(**cfg)) == 0


def test_singular_uv_matrix_rejected(L):
    # det = 1 + beta tau'/2 with beta = d tau' k2/h^2 + tau' mu^2/2; choose k2 < 0
    # so that det = 0 exactly: tau' = 0.5, h = 0.25 (n=8 on [-1,1)), d = 1:
    # beta = 0.5 k2 / 0.0625 = 8 k2 (mu = 0) and det = 1 + 8 k2 * 0.25 = 1 + 2 k2.
    cfg = good(dim=1, tau=1.0, kappa2=-0.5, mu=0.0)
    assert _init_status(cfg) == kgs.KGS_ESINGULAR
    assert "singular" in kgs.last_error(None)


def test_null_arguments(L):
    assert _init_status(None) == kgs.KGS_EINVAL
    assert _init_status(good(), ptr=None) == kgs.KGS_EINVAL
    h = ctypes.c_void_p()
    assert kgs.lib().kgs_init(ctypes.byref(good()), 1, 1, 1, 1, 7, None, ctypes.byref(h)) == \
        kgs.KGS_EINVAL
    assert kgs.lib().kgs_step(None, 1) == kgs.KGS_EINVAL
    e = ctypes.c_double()
    assert kgs.lib().kgs_energy(None, ctypes.byref(e)) == kgs.KGS_EINVAL
    assert kgs.lib().kgs_free(None) == kgs.KGS_OK


def test_required_bytes(L):
    # 3-D grids of n >= 96 run the ping-pong streaming kernel by default in
    # both precisions: two states
    cfg = good(dim=3, n=256)
    state = 8 * (256 ** 3 // 2) * 8
    assert 2 * state <= kgs.required_bytes(cfg) < 2 * state + (1 << 20)
    cfg32 = good(dim=3, n=256, precision=kgs.KGS_FP32)
    assert state <= kgs.required_bytes(cfg32) < state + (1 << 20)
    # below n = 96 they sweep in place: one state
    cfg64s = good(dim=3, n=64)
    small = 8 * (64 ** 3 // 2) * 8
    assert small <= kgs.required_bytes(cfg64s) < small + (1 << 20)
    # 2-D grids beyond the resident kernel run the tiled kernel (n < 2048) or
    # stream (n >= 2048), both between two states, in both precisions
    cfg2 = good(dim=2, n=1024)
    state2 = 8 * (1024 ** 2 // 2) * 8
    assert 2 * state2 <= kgs.required_bytes(cfg2) < 2 * state2 + (1 << 20)
    cfg2f = good(dim=2, n=1024, precision=kgs.KGS_FP32)
    assert state2 <= kgs.required_bytes(cfg2f) < state2 + (1 << 20)
    cfg2s = good(dim=2, n=64)  # resident: one state
    small2 = 8 * (64 ** 2 // 2) * 8
    assert small2 <= kgs.required_bytes(cfg2s) < small2 + (1 << 20)


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    # there is no fallback path: without the built library every entry of
    # the binding raises
    monkeypatch.setattr(kgs, "LIB_PATH", str(tmp_path / "libkgs.so"))
    monkeypatch.setattr(kgs, "_lib", None)
    with pytest.raises(ImportError):
        kgs.lib()
    with pytest.raises(ImportError):
        kgs.last_error(None)
    with pytest.raises(ImportError):
        kgs.kgs_step(None, 1)


def test_step_fields_rejects_before_device_use(L):
    # every check of kgs_step_fields comes before it looks up the device, so
    # fake pointers are never dereferenced
    f = kgs.lib().kgs_step_fields
    assert f(None, 1, 1, 1, 1, 1, None) == kgs.KGS_EINVAL
    assert f(ctypes.byref(good(n=7)), 1, 1, 1, 1, 1, None) == kgs.KGS_EODDN
    assert f(ctypes.byref(good()), None, 1, 1, 1, 1, None) == kgs.KGS_EINVAL
    assert f(ctypes.byref(good()), 1, 1, 1, 1, -1, None) == kgs.KGS_EINVAL
    # 3-D 130^3 float64: 8 planes of 130^3/2 values exceed the scratch area;
    # 128^3 float64 fills it exactly, and 164^3 float32 does not fit either
    assert f(ctypes.byref(good(dim=3, n=130)), 1, 1, 1, 1, 1, None) == kgs.KGS_ENOMEM
    assert "scratch" in kgs.last_error(None)
    assert 8 * (128 ** 3 // 2) * 8 == kgs.KGS_STEP_FIELDS_SCRATCH_BYTES
    assert f(ctypes.byref(good(dim=3, n=164, precision=kgs.KGS_FP32)), 1, 1, 1, 1, 1,
             None) == kgs.KGS_ENOMEM
