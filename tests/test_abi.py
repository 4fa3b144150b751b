"""The C-ABI library loads, exports every entry point include/rpr.h declares,
and rejects bad arguments before touching a device (no GPU needed)."""
import ctypes as C
import os
import re
import subprocess

import pytest

import paper_2411_06225_amd as rpr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_entry_points():
    src = open(os.path.join(ROOT, "include", "rpr.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)  # drop comments
    return sorted(set(re.findall(r"\b(rpr_[a-z0-9_]+)\s*\(", src)))


def test_header_and_binding_agree():
    assert declared_entry_points() == sorted(rpr.EXPORTED)


def test_library_exports_every_declared_symbol():
    out = subprocess.run(["nm", "-D", "--defined-only", rpr.LIB_PATH], capture_output=True, text=True, check=True)
    exported = set(re.findall(r"\sT\s(rpr_\w+)", out.stdout))
    assert set(declared_entry_points()) <= exported
    # nothing but the C ABI leaves the library
    assert exported == set(declared_entry_points())
    L = rpr.lib()
    for name in declared_entry_points():
        assert getattr(L, name) is not None


def test_version_string():
    assert rpr.lib().rpr_version().decode().startswith("rpr ")


def _prop(method=4, steps=10, threads=0):
    return rpr.rpr_propagator(method, threads, steps)


@pytest.mark.parametrize("kind,nx,ny,d,msg", [
    (0, 64, 1, 63, "d must equal"),
    (0, 64, 2, 128, "ny == 1"),
    (1, 8, 8, 100, "d must equal"),
    (9, 8, 8, 128, "kind"),
    (2, 0, 8, 0, "nx"),
])
def test_propagate_rejects_bad_problem(kind, nx, ny, d, msg):
    h = rpr.make_rhs(kind, nx, ny)
    st = rpr.lib().rpr_propagate(C.byref(h), d, C.byref(_prop()), 0, 1e-3, 1, 1 << 20, 1 << 30, None)
    assert st == rpr.RPR_ERR_INVALID_ARG
    assert msg in rpr.last_error()


def test_propagate_rejects_bad_propagator_and_overlap():
    h = rpr.make_rhs(0, 64)
    L = rpr.lib()
    assert L.rpr_propagate(C.byref(h), 64, C.byref(_prop(method=2)), 0, 1e-3, 1, 1 << 20, 1 << 30, None) == -1
    assert L.rpr_propagate(C.byref(h), 64, C.byref(_prop(steps=0)), 0, 1e-3, 1, 1 << 20, 1 << 30, None) == -1
    assert L.rpr_propagate(C.byref(h), 64, C.byref(_prop()), 5, 1e-3, 1, 1 << 20, 1 << 30, None) == -1
    assert L.rpr_propagate(C.byref(h), 64, C.byref(_prop(threads=100)), 0, 1e-3, 1, 1 << 20, 1 << 30, None) == -1
    assert "threads" in rpr.last_error()
    # the eighth-order method runs on the generic propagator only
    assert L.rpr_propagate(C.byref(h), 64, C.byref(_prop(method=8, threads=256)), 0, 1e-3, 1, 1 << 20, 1 << 30,
                           None) == rpr.RPR_ERR_UNSUPPORTED
    assert "generic" in rpr.last_error()
    # in and out overlapping
    assert L.rpr_propagate(C.byref(h), 64, C.byref(_prop()), 0, 1e-3, 2, 4096, 4096 + 512, None) == -1
    assert "overlap" in rpr.last_error()


@pytest.mark.parametrize("kind,nx,ny,nz,d,msg", [
    (rpr.RPR_BRUSS3D, 8, 8, 0, 128, "nz"),            # the 3D system needs nz >= 1
    (rpr.RPR_BRUSS3D, 8, 8, 4, 2 * 8 * 8, "d must equal"),
    (rpr.RPR_BRUSS2D, 8, 8, 2, 2 * 8 * 8 * 2, "nz"),  # 2D systems take nz 0 or 1
])
def test_propagate_rejects_bad_3d_problem(kind, nx, ny, nz, d, msg):
    h = rpr.make_rhs(kind, nx, ny, nz=nz)
    st = rpr.lib().rpr_propagate(C.byref(h), d, C.byref(_prop()), 0, 1e-3, 1, 1 << 20, 1 << 30, None)
    assert st == rpr.RPR_ERR_INVALID_ARG
    assert msg in rpr.last_error()


@pytest.mark.parametrize("threads", [256, 512, 1024])
def test_3d_system_runs_on_the_generic_propagator_only(threads):
    h = rpr.make_rhs(rpr.RPR_BRUSS3D, 8, 8, nz=8)
    st = rpr.lib().rpr_propagate(C.byref(h), 2 * 8 ** 3, C.byref(_prop(threads=threads)), 0, 1e-3, 1, 1 << 20,
                                 1 << 30, None)
    assert st == rpr.RPR_ERR_UNSUPPORTED
    assert "generic" in rpr.last_error()


@pytest.mark.parametrize("kind,nx,ny,prec,threads", [(1, 13, 9, 0, 512), (0, 128, 1, 0, 512), (1, 32, 32, 1, 512),
                                                     (2, 128, 128, 0, 512), (0, 128, 1, 0, 256), (0, 4096, 1, 1, 256)])
def test_propagate_rejects_work_group_size_without_kernel(kind, nx, ny, prec, threads):
    # 512-thread kernels exist for the 64 x 64 grids only, the tiled form
    # (256) for 2D grids only; decided on the host
    h = rpr.make_rhs(kind, nx, ny)
    d = rpr.nspecies(kind) * nx * ny
    st = rpr.lib().rpr_propagate(C.byref(h), d, C.byref(_prop(threads=threads)), prec, 1e-3, 1, 1 << 20, 1 << 30,
                                 None)
    assert st == rpr.RPR_ERR_UNSUPPORTED


def test_plan_create_rejects_bad_options():
    h = rpr.make_rhs(0, 32)
    F, G = _prop(4, 10), _prop(1, 2)
    net = rpr.rpr_randnet(10, 0, 1e-6, 0.0)
    L = rpr.lib()
    handle = C.c_void_p()

    def create(d=32, t0=0.0, tN=1.0, N=4, tol=1e-6, net_=net, opt=None):
        opt = opt or rpr.rpr_options(0, 0, 0, 0, 0, 0, 0, 0)
        return L.rpr_plan_create(C.byref(handle), C.byref(h), d, t0, tN, N, C.byref(F), C.byref(G), tol,
                                 C.byref(net_), None, None, 0, C.byref(opt))

    assert create(N=0) == -1
    assert create(tN=0.0) == -1
    assert create(tol=float("nan")) == -1
    assert create(net_=rpr.rpr_randnet(0, 0, 1e-6, 0.0)) == -1
    assert create(net_=rpr.rpr_randnet(10, 0, 0.0, 0.0)) == -1
    assert create(net_=rpr.rpr_randnet(10, 7, 1e-6, 0.0)) == -1
    assert create(opt=rpr.rpr_options(3, 0, 0, 0, 0, 0, 0, 0)) == -1
    assert create(opt=rpr.rpr_options(0, 0, 9, 0, 0, 0, 0, 0)) == -1
    assert create(opt=rpr.rpr_options(0, 0, 0, 0, 5, 0, 0, 0)) == -1
    assert create(opt=rpr.rpr_options(0, 0, 0, 0, 0, 2, 0, 0)) == -1
    assert create(opt=rpr.rpr_options(0, 0, 0, 0, 0, 0, 3, 0)) == -1
    assert create(opt=rpr.rpr_options(0, 0, 0, 0, 0, 0, 0, 2)) == -1
    assert create(opt=rpr.rpr_options(0, 3, 0, 0, 0, 0, 0, 0)) == -1
    assert create(opt=rpr.rpr_options(0, 0, 0, 0, 0, 0, 0, 0, -1, 0)) == -1  # chain_wgs
    assert create(opt=rpr.rpr_options(0, 0, 0, 0, 0, 0, 0, 0, 0, 3)) == -1  # sweep_form
    assert "sweep_form" in rpr.last_error()
    # nearest-neighbour correction: 1 <= m_nn <= 32, reserved field zero
    nn = rpr.rpr_options(0, rpr.RPR_CORR_RANDNET_NN, 0, 0, 0, 0, 0, 0)
    assert create(net_=rpr.rpr_randnet(10, 0, 1e-6, 0.0, 0, 0), opt=nn) == -1
    assert create(net_=rpr.rpr_randnet(10, 0, 1e-6, 0.0, 33, 0), opt=nn) == -1
    assert create(net_=rpr.rpr_randnet(10, 0, 1e-6, 0.0, 4, 1), opt=nn) == -1
    assert handle.value is None


def test_batch_checks_nearest_neighbour_count():
    h = (rpr.rpr_rhs * 1)(rpr.make_rhs(0, 32))
    F, G = (rpr.rpr_propagator * 1)(_prop(4, 10)), (rpr.rpr_propagator * 1)(_prop(1, 2))
    net = (rpr.rpr_randnet * 1)(rpr.rpr_randnet(10, 0, 1e-6, 0.0, 0, 0))
    d, N = (C.c_int32 * 1)(32), (C.c_int32 * 1)(4)
    t0, tN, tol = (C.c_double * 1)(0.0), (C.c_double * 1)(1.0), (C.c_double * 1)(1e-6)
    opt = rpr.rpr_options(0, rpr.RPR_CORR_RANDNET_NN, 0, 0, 0, 0, 0, 0)
    handle = C.c_void_p()
    st = rpr.lib().rpr_plan_create_batch(C.byref(handle), 1, h, d, t0, tN, N, F, G, tol, net, None, None, 0,
                                         C.byref(opt))
    assert st == rpr.RPR_ERR_INVALID_ARG
    assert handle.value is None


def test_destroy_accepts_null():
    assert rpr.lib().rpr_plan_destroy(None) == rpr.RPR_OK


def test_building_blocks_reject_bad_sizes():
    L = rpr.lib()
    assert L.rpr_randnet_features(0, 4, 1, 0, 1.0, 1, 2, 3, 4, None) == -1
    assert L.rpr_randnet_features(4, 4, 1, 0, 0.0, 1, 2, 3, 4, None) == -1
    assert L.rpr_ridge_fit(4, 4, 1, 1, 2, 0.0, 3, None) == -1
    assert L.rpr_ridge_fit(4000, 4, 1, 1, 2, 1e-3, 3, None) == -1
    assert L.rpr_uniform_pm1(0, 0, -1, 1, None) == -1
    # zero-sized work is a no-op that needs no device
    assert L.rpr_randnet_readout(4, 4, 0, 1, 2, 3, None) == rpr.RPR_OK


def test_strict_stability_check_rejects_unstable_coarse_solver_before_any_device_call():
    # heat-like Brusselator (A = B = 0) on 32 x 32 cells of (-1, 1)^2, D = 0.1:
    # rho_r = D (4/dx^2 + 4/dy^2) + 1 = 0.1 * 8 * 256 + 1 = 205.8; one forward
    # Euler step over a slice of 0.25 is far outside |1 + z| <= 1
    h = rpr.make_rhs(rpr.RPR_BRUSS2D, 32, 32, params=(0.0, 0.0, 0.1, 0.1))
    F, G = _prop(4, 200), _prop(1, 1)
    net = rpr.rpr_randnet(10, 0, 1e-6, 0.0, 0, 0)
    handle = C.c_void_p()
    strict = rpr.rpr_options(0, 0, 0, 0, 0, 0, 0, 1)
    st = rpr.lib().rpr_plan_create(C.byref(handle), C.byref(h), 2 * 32 * 32, 0.0, 1.0, 4, C.byref(F), C.byref(G),
                                   1e-6, C.byref(net), None, None, 0, C.byref(strict))
    assert st == rpr.RPR_ERR_UNSTABLE
    assert "stability" in rpr.last_error()
    assert handle.value is None


def test_stability_ratio_closed_forms():
    # forward Euler on the periodic heat equation: dt_max = 2 / (D (4/dx^2 + 4/dy^2) + B + 1)
    # with A = B = 0: 2 / (0.1 * 2048 + 1)
    h = rpr.make_rhs(rpr.RPR_BRUSS2D, 32, 32, params=(0.0, 0.0, 0.1, 0.05))
    rho = 0.1 * 8 * 256 + 1.0
    assert rpr.rpr_stability(h, 2048, 1, 1, 1e-3, 0.0) == pytest.approx(1e-3 * rho / 2, rel=1e-15)
    assert rpr.rpr_stability(h, 2048, 4, 1, 1e-3, 0.0) == pytest.approx(1e-3 * rho / 2.78, rel=1e-15)
    # Burgers: rho_r = 4 nu / dx^2, rho_i = umax / dx; forward Euler needs
    # dt <= 2 / rho_r and dt <= rho_r / (2 rho_i^2) (= 2 nu / umax^2)
    hb = rpr.make_rhs(rpr.RPR_BURGERS1D, 128, 1, params=(0.01,))
    dx = 2.0 / 128
    rr, ri = 4 * 0.01 / dx ** 2, 1.5 / dx
    dt = 5.0 / 16 / 40
    want = max(dt * rr / 2, dt * 2 * ri * ri / rr)
    assert rpr.rpr_stability(hb, 128, 1, 40, dt, 1.5) == pytest.approx(want, rel=1e-14)
    assert want == pytest.approx(dt * 1.5 ** 2 / (2 * 0.01), rel=1e-14)
    # the stated Burgers workload's G (4 steps per slice) is unstable, 40 steps are not
    assert rpr.rpr_stability(hb, 128, 1, 4, 5.0 / 16 / 4, 1.5) > 1
    assert rpr.rpr_stability(hb, 128, 1, 40, 5.0 / 16 / 40, 1.5) < 1
    # shallow water, 192 x 192 on [0, 1]^2: rho_r = 2 a (1/dx + 1/dy)
    hs = rpr.make_rhs(rpr.RPR_SWE2D, 192, 192, domain=(0.0, 1.0, 0.0, 1.0), params=(9.81,))
    a = (9.81 * 1.1) ** 0.5
    r = rpr.rpr_stability(hs, 3 * 192 * 192, 1, 8, 1.0 / 256 / 8, 1.1, a)
    assert r == pytest.approx(1.0 / 256 / 8 * 2 * a * 384 / 2, rel=1e-14)
    assert r < 1
    # bad arguments
    with pytest.raises(rpr.RprError):
        rpr.rpr_stability(hs, 3 * 192 * 192, 1, 8, 1e-3, -1.0)


def test_tuning_table_set_get_and_remove():
    # host-only table of launch shapes: no device is touched
    key = "prop:3:96x80:4:4:v"
    assert rpr.rpr_tune_get(key) is None
    try:
        rpr.rpr_tune_set(key, 5)
        assert rpr.rpr_tune_get(key) == 5
        rpr.rpr_tune_set(key, 2)
        assert rpr.rpr_tune_get(key) == 2
    finally:
        rpr.rpr_tune_set(key, -1)
    assert rpr.rpr_tune_get(key) is None
    L = rpr.lib()
    assert L.rpr_tune_set(b"", 1) == rpr.RPR_ERR_INVALID_ARG
    assert L.rpr_tune_set(None, 1) == rpr.RPR_ERR_INVALID_ARG
    assert L.rpr_tune_get(b"prop:none", None) == rpr.RPR_ERR_INVALID_ARG
    v = C.c_int32(0)
    assert L.rpr_tune_get(b"prop:none", C.byref(v)) == rpr.RPR_ERR_INVALID_ARG
    assert "no entry" in rpr.last_error()


def test_tile_shape_names():
    swe32 = rpr.tile_shapes(rpr.RPR_SWE2D, rpr.RPR_MIXED)
    swe64 = rpr.tile_shapes(rpr.RPR_SWE2D, rpr.RPR_FP64)
    assert swe32[0] == "R5NW8" and swe64[0] == "R4NW8"
    assert any(s.startswith("rows:C3") for s in swe32) and any(s.startswith("rows:C3") for s in swe64)
    assert len(set(swe32)) == len(swe32) and len(set(swe64)) == len(swe64)
    assert rpr.tile_shapes(rpr.RPR_DIFFREACT2D, rpr.RPR_FP64)[0] == "FY32NT512"
    assert rpr.tile_shapes(rpr.RPR_BURGERS1D, rpr.RPR_FP64) == ["default"]
    L = rpr.lib()
    assert L.rpr_tile_shape_name(rpr.RPR_SWE2D, rpr.RPR_MIXED, len(swe32)) is None
    assert L.rpr_tile_shape_name(rpr.RPR_SWE2D, rpr.RPR_MIXED, -1) is None
