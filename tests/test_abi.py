"""C ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and host-side validation rejects bad arguments before any
device call (include/bfm.h)."""
import ctypes
import os
import re

import pytest

from paper_1905_12154_amd import bfm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bfm.h")


def declared_symbols():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bfm_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = bfm.lib()
    names = declared_symbols()
    assert len(names) >= 10
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(bfm.EXPORTED)
    assert L.bfm_version().decode().startswith("bfm-gfx950")


def _params(shape, dtype=bfm.BFM_F32):
    p = bfm.Params()
    shp = (ctypes.c_int32 * 3)(*(list(shape) + [1] * (3 - len(shape))))
    st = bfm.lib().bfm_params_init(ctypes.byref(p), len(shape), shp, dtype)
    return st, p


@pytest.mark.parametrize("shape", [(64, 64), (384, 1024), (4096, 4096), (96, 48, 64), (4, 6)])
def test_params_defaults_are_paper_constants(shape):
    st, p = _params(shape)
    assert st == bfm.BFM_OK
    assert (p.sigma_min, p.beta1, p.beta2, p.alpha1, p.alpha2) == (0.01, 0.25, 0.75, 1.25, 0.8)
    assert p.sigma0 == 0.0 and p.tol == 0.0
    assert p.method == bfm.METHODS["bfm"] == 0


@pytest.mark.parametrize("shape", [(5, 8), (64, 8192), (2, 64), (64,), (7, 7, 7), (64, 64, 64, 64)])
def test_bad_shapes_rejected(shape):
    if len(shape) in (1, 4):
        p = bfm.Params()
        shp = (ctypes.c_int32 * 3)(64, 64, 64)
        st = bfm.lib().bfm_params_init(ctypes.byref(p), len(shape), shp, 0)
    else:
        st, p = _params(shape)
    assert st == bfm.BFM_EINVAL
    assert "n" in bfm.lib().bfm_last_error().decode()
    h = ctypes.c_void_p()
    assert bfm.lib().bfm_plan_create(ctypes.byref(p), ctypes.byref(h)) == bfm.BFM_EINVAL
    assert not h.value


@pytest.mark.parametrize("field,value", [("dtype", 7), ("beta1", 0.9), ("alpha1", 0.5), ("alpha2", 1.5),
                                         ("sigma_min", 0.0), ("tol", -1.0), ("check_every", 0),
                                         ("max_iters", -3), ("sigma0", float("nan")), ("method", 2),
                                         ("method", -1)])
def test_bad_parameters_rejected(field, value):
    st, p = _params((32, 32))
    setattr(p, field, value)
    h = ctypes.c_void_p()
    assert bfm.lib().bfm_plan_create(ctypes.byref(p), ctypes.byref(h)) == bfm.BFM_EINVAL
    assert bfm.lib().bfm_last_error().decode()


def test_workspace_size_and_errors_before_launch():
    plan = bfm.Plan((64, 48), dtype="float64")
    assert plan.ws_bytes >= 3 * 64 * 48 * 8
    L = bfm.lib()
    res = bfm.Result()
    dummy = ctypes.c_void_p(0x1000)
    mu, nu, phi, psi = (ctypes.c_void_p(a) for a in (0x1000, 0x1100, 0x1200, 0x1300))
    # null workspace -> EWORKSPACE (validated before any device call)
    st = L.bfm_solve(plan.handle, mu, nu, None, phi, psi, None, None, plan.ws_bytes, None, ctypes.byref(res))
    assert st == bfm.BFM_EWORKSPACE
    # misaligned
    st = L.bfm_solve(plan.handle, mu, nu, None, phi, psi, None, ctypes.c_void_p(0x1010), plan.ws_bytes, None,
                     ctypes.byref(res))
    assert st == bfm.BFM_EWORKSPACE
    # too small
    st = L.bfm_solve(plan.handle, mu, nu, None, phi, psi, None, ctypes.c_void_p(0x10000), plan.ws_bytes - 1, None,
                     ctypes.byref(res))
    assert st == bfm.BFM_EWORKSPACE
    # null densities / aliased outputs -> EINVAL
    assert L.bfm_solve(plan.handle, None, nu, None, phi, psi, None, ctypes.c_void_p(0x10000), plan.ws_bytes,
                       None, ctypes.byref(res)) == bfm.BFM_EINVAL
    assert L.bfm_solve(plan.handle, mu, nu, None, phi, phi, None, ctypes.c_void_p(0x10000), plan.ws_bytes,
                       None, ctypes.byref(res)) == bfm.BFM_EINVAL
    assert L.bfm_solve(None, dummy, dummy, None, dummy, dummy, None, None, 0, None, None) == bfm.BFM_EINVAL
    assert L.bfm_ctransform(plan.handle, None, dummy, None, 0, None) == bfm.BFM_EINVAL
    assert L.bfm_grad(plan.handle, dummy, dummy, float("inf"), None, None, ctypes.c_void_p(0x10000),
                      plan.ws_bytes, None) == bfm.BFM_EINVAL
    L.bfm_plan_workspace_bytes(None, None)
    assert "NULL" in L.bfm_last_error().decode()


@pytest.mark.parametrize("value", [1.0, 1.04, 8.5, float("nan"), float("inf")])
def test_bad_cost_exponent_rejected(value):
    st, p = _params((32, 32))
    assert tuple(p.power) == (2.0, 2.0, 2.0)
    p.power[1] = value
    h = ctypes.c_void_p()
    assert bfm.lib().bfm_plan_create(ctypes.byref(p), ctypes.byref(h)) == bfm.BFM_EINVAL
    assert "power[1]" in bfm.lib().bfm_last_error().decode()
    # the exponent of an axis beyond ndim is not read
    st, p = _params((32, 32))
    p.power[2] = value
    assert bfm.lib().bfm_plan_create(ctypes.byref(p), ctypes.byref(h)) == bfm.BFM_OK
    bfm.lib().bfm_plan_destroy(h)


def test_plan_python_validation():
    plan = bfm.Plan((32, 32))
    with pytest.raises(TypeError):
        plan.ctransform(__import__("torch").zeros(32, 32))
    with pytest.raises(bfm.BFMError):
        bfm.Plan((31, 32))
    with pytest.raises(ValueError):
        bfm.Plan((32, 32), method="newton")
    assert bfm.Plan((32, 32), method="ga").params.method == 1


def test_header_is_plain_c():
    """The boundary header compiles as C99 (no C++ types cross the ABI)."""
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no C compiler")
    hdr = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "bfm.h")
    r = subprocess.run([gcc, "-std=c99", "-Wall", "-Wextra", "-Werror", "-fsyntax-only", "-x", "c", hdr],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_noalloc_rejects_plans_above_its_static_scratch():
    """bfm_solve_noalloc refuses a plan whose workspace exceeds its 64 MiB
    static array before any device call; plans that fit are not refused by
    that check (float32 2048^2 and float64 1536^2 fit, float32 4096^2 does
    not)."""
    L = bfm.lib()
    res = bfm.Result()
    d = [ctypes.c_void_p(0x1000 + 0x100 * k) for k in range(5)]
    for shape, dt, fits in (((4096, 4096), "float32", False), ((2048, 2048), "float64", False),
                            ((2048, 2048), "float32", True), ((1536, 1536), "float64", True)):
        plan = bfm.Plan(shape, dtype=dt)
        assert (plan.ws_bytes <= 64 << 20) == fits
        if not fits:
            st = L.bfm_solve_noalloc(plan.handle, d[0], d[1], None, d[2], d[3], None, None, ctypes.byref(res))
            assert st == bfm.BFM_EWORKSPACE
            assert "static array" in L.bfm_last_error().decode()
    assert L.bfm_solve_noalloc(None, d[0], d[1], None, d[2], d[3], None, None, ctypes.byref(res)) == bfm.BFM_EINVAL


def test_grad_batched_validation_before_any_launch():
    L = bfm.lib()
    plan = bfm.Plan((32, 32), dtype="float64")
    VP = ctypes.c_void_p * 2
    ws_ok = [0x100000, 0x100000 + ((plan.ws_bytes + 255) // 256) * 256]
    f = VP(0x1000, 0x2000)
    plans = VP(plan.handle.value, plan.handle.value)
    sizes = (ctypes.c_size_t * 2)(plan.ws_bytes, plan.ws_bytes)
    ones = (ctypes.c_double * 2)(1.0, 1.0)
    assert L.bfm_grad_batched(0, plans, f, f, ones, f, f, VP(*ws_ok), sizes, None) == bfm.BFM_EINVAL
    assert L.bfm_grad_batched(2, plans, None, f, ones, f, f, VP(*ws_ok), sizes, None) == bfm.BFM_EINVAL
    bad = (ctypes.c_double * 2)(1.0, float("nan"))
    assert L.bfm_grad_batched(2, plans, f, f, bad, f, f, VP(*ws_ok), sizes, None) == bfm.BFM_EINVAL
    assert "scale" in L.bfm_last_error().decode()
    shared = VP(ws_ok[0], ws_ok[0])
    assert L.bfm_grad_batched(2, plans, f, f, ones, f, f, shared, sizes, None) == bfm.BFM_EINVAL
    small = (ctypes.c_size_t * 2)(plan.ws_bytes, plan.ws_bytes - 1)
    assert L.bfm_grad_batched(2, plans, f, f, ones, f, f, VP(*ws_ok), small, None) == bfm.BFM_EWORKSPACE


def test_deposit_grid_setting_and_validation():
    # built-in: one workgroup per source tile (16 x 32 in 2D, 8^3 in 3D), at most 2048
    plan = bfm.Plan((64, 64))
    assert plan.deposit_grid() == (64 // 16) * (64 // 32)
    assert bfm.Plan((384, 256)).deposit_grid() == (384 // 16) * (256 // 32)
    assert bfm.Plan((4096, 4096)).deposit_grid() == 2048
    assert bfm.Plan((64, 64, 64)).deposit_grid() == 512
    for bad in (7, 4, -8, 8200, 16384):
        with pytest.raises(bfm.BFMError) as e:
            plan.set_deposit_grid(bad)
        assert e.value.status == bfm.BFM_EINVAL
    plan.set_deposit_grid(8192)
    assert plan.deposit_grid() == 8192
    plan.set_deposit_grid(0)
    assert plan.deposit_grid() == 8
