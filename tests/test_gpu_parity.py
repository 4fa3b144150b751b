"""GPU parity: every building block of librpr against the CPU oracle, through the C ABI.

Sizes span several work-group tiles and ragged tails; the workload shapes
(64 x 64 diffusion-reaction, 64 x 64 Brusselator, Burgers d = 128 and 4096)
use the kernel instances the benchmark runs.

Tolerances (relative to the largest magnitude of the reference):
  - propagators, FP64: 1e-12.  Both sides evaluate the same formulas; they
    differ only in rounding (reciprocal multiplies vs divides, fused
    multiply-adds), a few ulps per step that do not grow on these stable runs.
  - propagators, FP32 states: 2e-5 after the given number of steps (unit
    roundoff 6e-8 times the step count, bounded by the test's measurement).
  - features and readout: 1e-13 (a sum of d or M products).
  - ridge readout: max(1e-12, 10 kappa 2^-53), kappa = cond(Phi^T Phi + lambda I),
    the forward-error bound of a backward-stable Cholesky solve.
  - generator: bitwise.
"""
import ctypes as C
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2411_06225_amd as rpr  # noqa: E402


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


def rel_err(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


# (kind, nx, ny, domain, params, steps, dt, method) -- stable step sizes
PROP_CASES = [
    ("burgers_d128", rpr.RPR_BURGERS1D, 128, 1, (-1, 1, -1, 1), (0.01,), 300, 1.5e-4, 4),
    ("burgers_d100_ragged", rpr.RPR_BURGERS1D, 100, 1, (-1, 1, -1, 1), (0.02,), 300, 1.5e-4, 4),
    ("burgers_d1000", rpr.RPR_BURGERS1D, 1000, 1, (-1, 1, -1, 1), (0.002,), 100, 2e-5, 4),
    ("burgers_d4096", rpr.RPR_BURGERS1D, 4096, 1, (-1, 1, -1, 1), (0.001,), 50, 2e-6, 4),
    ("burgers_rk1", rpr.RPR_BURGERS1D, 128, 1, (-1, 1, -1, 1), (0.01,), 40, 2e-3, 1),
    ("diffreact_64x64", rpr.RPR_DIFFREACT2D, 64, 64, (-1, 1, -1, 1), (1e-3, 5e-3, 5e-3), 200, 7.8125e-5, 4),
    ("diffreact_13x9", rpr.RPR_DIFFREACT2D, 13, 9, (-1, 1, -1, 1), (1e-3, 5e-3, 5e-3), 200, 1e-3, 4),
    ("diffreact_32x32_rk1", rpr.RPR_DIFFREACT2D, 32, 32, (-1, 1, -1, 1), (1e-3, 5e-3, 5e-3), 20, 0.01, 1),
    ("diffreact_40x70", rpr.RPR_DIFFREACT2D, 40, 70, (-1, 1, -1, 1), (1e-3, 5e-3, 5e-3), 100, 1e-3, 4),
    ("bruss_64x64", rpr.RPR_BRUSS2D, 64, 64, (-1, 1, -1, 1), (1.0, 3.0, 0.02, 0.01), 200, 2e-4, 4),
    ("bruss_20x16", rpr.RPR_BRUSS2D, 20, 16, (-1, 1, -1, 1), (1.0, 3.0, 0.02, 0.01), 200, 1e-3, 4),
    ("swe_24x16", rpr.RPR_SWE2D, 24, 16, (0, 1, 0, 1), (9.81,), 200, 5e-4, 4),
    ("swe_8x40_rk1", rpr.RPR_SWE2D, 8, 40, (0, 1, 0, 1), (9.81,), 50, 2e-4, 1),
]


def initial_state(kind, nx, ny, rng):
    nc = nx * ny
    if kind == rpr.RPR_BURGERS1D:
        x = -1 + 2 * np.arange(nx) / nx
        return 0.5 * np.sin(np.pi * x) + 0.3 * np.cos(3 * np.pi * x) + 0.05 * rng.standard_normal(nx)
    if kind == rpr.RPR_DIFFREACT2D:
        return rng.standard_normal(2 * nc)
    if kind == rpr.RPR_BRUSS2D:
        return np.concatenate([1 + 0.1 * rng.uniform(-1, 1, nc), 3 + 0.1 * rng.uniform(-1, 1, nc)])
    h = 1 + 0.1 * rng.random(nc)
    return np.concatenate([h, 0.05 * rng.standard_normal(nc), 0.05 * rng.standard_normal(nc)])


@pytest.mark.parametrize("case", PROP_CASES, ids=[c[0] for c in PROP_CASES])
def test_propagate_fp64_matches_oracle(orc, case):
    name, kind, nx, ny, dom, params, steps, dt, method = case
    rng = np.random.default_rng(abs(hash(name)) % 2 ** 32)
    d = rpr.nspecies(kind) * nx * ny
    n = 3
    X = np.stack([initial_state(kind, nx, ny, rng) for _ in range(n)])
    pb = orc.problem(kind, nx, ny, dom, params)
    ref = orc.propagate_many(pb, method, steps, dt, X)
    xin, xout = dev(X), torch.empty((n, d), dtype=torch.float64, device="cuda")
    rpr.rpr_propagate(rpr.make_rhs(kind, nx, ny, dom, params), d, method, steps, rpr.RPR_FP64, dt, n, xin, xout)
    got = host(xout)
    print(name, "rel err %.2e" % rel_err(got, ref))
    assert np.all(np.isfinite(got))
    assert rel_err(got, ref) <= 1e-12


@pytest.mark.parametrize("case", [c for c in PROP_CASES if c[0] in ("burgers_d128", "diffreact_64x64", "bruss_64x64",
                                                                    "swe_24x16", "diffreact_13x9")],
                         ids=lambda c: c[0])
def test_propagate_fp32_states_close_to_fp64_oracle(orc, case):
    name, kind, nx, ny, dom, params, steps, dt, method = case
    rng = np.random.default_rng(7)
    d = rpr.nspecies(kind) * nx * ny
    X = initial_state(kind, nx, ny, rng)[None]
    pb = orc.problem(kind, nx, ny, dom, params)
    ref = orc.propagate_many(pb, method, steps, dt, X)
    xin, xout = dev(X, torch.float32), torch.empty((1, d), dtype=torch.float32, device="cuda")
    rpr.rpr_propagate(rpr.make_rhs(kind, nx, ny, dom, params), d, method, steps, rpr.RPR_MIXED, dt, 1, xin, xout)
    err = rel_err(host(xout), ref)
    print(name, "fp32 rel err %.2e" % err)
    assert err <= 2e-5


@pytest.mark.parametrize("case", [c for c in PROP_CASES if c[0] in ("diffreact_64x64", "bruss_64x64")],
                         ids=lambda c: c[0])
@pytest.mark.parametrize("threads", [512, 1024])
@pytest.mark.parametrize("prec", [rpr.RPR_FP64, rpr.RPR_MIXED], ids=["fp64", "fp32"])
def test_propagate_every_work_group_size(orc, case, threads, prec):
    """Both kernel instances of the 64 x 64 grids (strips of 8 rows on 512
    threads, of 4 rows on 1024), RK4 and forward Euler."""
    name, kind, nx, ny, dom, params, steps, dt, method = case
    rng = np.random.default_rng(11)
    d = rpr.nspecies(kind) * nx * ny
    X = np.stack([initial_state(kind, nx, ny, rng) for _ in range(2)])
    pb = orc.problem(kind, nx, ny, dom, params)
    h = rpr.make_rhs(kind, nx, ny, dom, params)
    dtype = torch.float64 if prec == rpr.RPR_FP64 else torch.float32
    for meth, st in ((method, steps), (1, 20)):
        ref = orc.propagate_many(pb, meth, st, dt, X)
        xin, xout = dev(X, dtype), torch.empty((2, d), dtype=dtype, device="cuda")
        rpr.rpr_propagate(h, d, meth, st, prec, dt, 2, xin, xout, threads=threads)
        err = rel_err(host(xout), ref)
        print(name, threads, meth, "rel err %.2e" % err)
        assert err <= (1e-12 if prec == rpr.RPR_FP64 else 2e-5)


TILED_CASES = [c for c in PROP_CASES if c[1] != rpr.RPR_BURGERS1D] + [
    ("swe_96x80", rpr.RPR_SWE2D, 96, 80, (0, 1, 0, 1), (9.81,), 30, 2e-4, 4),
    ("diffreact_130x70", rpr.RPR_DIFFREACT2D, 130, 70, (-1, 1, -1, 1), (1e-3, 5e-3, 5e-3), 20, 2e-4, 4),
    ("bruss_80x33_rk1", rpr.RPR_BRUSS2D, 80, 33, (-1, 1, -1, 1), (1.0, 3.0, 0.02, 0.01), 30, 1e-4, 1),
    ("bruss_70x37", rpr.RPR_BRUSS2D, 70, 37, (-1, 1, -1, 1), (1.0, 3.0, 0.02, 0.01), 30, 1e-4, 4),
    ("diffreact_67x17", rpr.RPR_DIFFREACT2D, 67, 17, (-1, 1, -1, 1), (1e-3, 5e-3, 5e-3), 30, 2e-4, 4),
    # shallow water, one pass per RK4 step: 56-column tiles (130 = 56 + 56 + 18,
    # 57 = 56 + 1), several tile rows, the smallest grid the 4-cell mirror halo
    # allows (4 cells each way), and the 192 x 192 grid (4 x 6 / 4 x 8 tiles)
    ("swe_130x70", rpr.RPR_SWE2D, 130, 70, (0, 1, 0, 1), (9.81,), 30, 2e-4, 4),
    ("swe_57x33", rpr.RPR_SWE2D, 57, 33, (0, 1, 0, 1), (9.81,), 30, 2e-4, 4),
    ("swe_4x4", rpr.RPR_SWE2D, 4, 4, (0, 1, 0, 1), (9.81,), 30, 2e-3, 4),
    ("swe_5x90", rpr.RPR_SWE2D, 5, 90, (0, 1, 0, 1), (9.81,), 30, 2e-4, 4),
    ("swe_192x192", rpr.RPR_SWE2D, 192, 192, (0, 1, 0, 1), (9.81,), 10, 2e-5, 4),
]


@pytest.mark.parametrize("case", TILED_CASES, ids=[c[0] for c in TILED_CASES])
@pytest.mark.parametrize("prec", [rpr.RPR_FP64, rpr.RPR_MIXED], ids=["fp64", "fp32"])
def test_tiled_propagate_matches_oracle(orc, case, prec):
    """The tiled form (states in memory, one pass over 64 x 16-cell tiles
    per RK stage, or per RK4 step with a 4-cell halo for the Laplacian
    systems) on grids with full and ragged tiles, tails of a few cells, walls
    and periodic boundaries, several states per launch."""
    name, kind, nx, ny, dom, params, steps, dt, method = case
    rng = np.random.default_rng(abs(hash(name)) % 2 ** 32 + 1)
    d = rpr.nspecies(kind) * nx * ny
    X = np.stack([initial_state(kind, nx, ny, rng) for _ in range(3)])
    pb = orc.problem(kind, nx, ny, dom, params)
    ref = orc.propagate_many(pb, method, steps, dt, X)
    dtype = torch.float64 if prec == rpr.RPR_FP64 else torch.float32
    xin, xout = dev(X, dtype), torch.empty((3, d), dtype=dtype, device="cuda")
    rpr.rpr_propagate(rpr.make_rhs(kind, nx, ny, dom, params), d, method, steps, prec, dt, 3, xin, xout, threads=256)
    err = rel_err(host(xout), ref)
    print(name, "tiled", "fp64" if prec == rpr.RPR_FP64 else "fp32", "rel err %.2e" % err)
    assert np.all(np.isfinite(host(xout)))
    assert err <= (1e-12 if prec == rpr.RPR_FP64 else 2e-5)


SHAPE_GRIDS = [(rpr.RPR_SWE2D, 192, 192, 4), (rpr.RPR_SWE2D, 96, 80, 30), (rpr.RPR_SWE2D, 57, 33, 30),
               (rpr.RPR_SWE2D, 4, 4, 30), (rpr.RPR_SWE2D, 130, 70, 30), (rpr.RPR_SWE2D, 126, 29, 31),
               (rpr.RPR_DIFFREACT2D, 130, 70, 20), (rpr.RPR_BRUSS2D, 70, 37, 21)]


@pytest.mark.parametrize("kind,nx,ny,steps", SHAPE_GRIDS, ids=lambda v: str(v))
@pytest.mark.parametrize("prec", [rpr.RPR_FP64, rpr.RPR_MIXED], ids=["fp64", "fp32"])
def test_every_tile_shape_matches_oracle(orc, kind, nx, ny, steps, prec):
    """Each tile shape of the one-pass RK4 kernels, pinned through the
    autotuner's table: the 56-column tiles with a 4-cell halo and the
    full-row form (whole rows per wavefront, C cells per lane; 192 = 64 x 3
    fills every lane, 57 and 126 leave lanes past the east wall, 4 x 4 puts
    both walls on one lane), on grids each shape serves; a shape that does
    not serve the grid is refused."""
    rng = np.random.default_rng(nx * 1000 + ny)
    d = rpr.nspecies(kind) * nx * ny
    dom = (0, 1, 0, 1) if kind == rpr.RPR_SWE2D else (-1, 1, -1, 1)
    params = {rpr.RPR_SWE2D: (9.81,), rpr.RPR_DIFFREACT2D: (1e-3, 5e-3, 5e-3),
              rpr.RPR_BRUSS2D: (1.0, 3.0, 0.02, 0.01)}[kind]
    dt = 2e-5 if nx >= 192 else 2e-4
    X = np.stack([initial_state(kind, nx, ny, rng) for _ in range(3)])
    ref = orc.propagate_many(orc.problem(kind, nx, ny, dom, params), 4, steps, dt, X)
    h = rpr.make_rhs(kind, nx, ny, dom, params)
    key = rpr.prop_tune_key(kind, nx, ny, prec, 4) + ":v"
    dtype = torch.float64 if prec == rpr.RPR_FP64 else torch.float32
    served = 0
    try:
        for v, name in enumerate(rpr.tile_shapes(kind, prec)):
            rpr.rpr_tune_set(key, v)
            xin, xout = dev(X, dtype), torch.zeros((3, d), dtype=dtype, device="cuda")
            st = rpr.lib().rpr_propagate(C.byref(h), d, C.byref(rpr.rpr_propagator(4, 256, steps)), prec, dt, 3,
                                         xin.data_ptr(), xout.data_ptr(), None)
            rows = name.startswith("rows:")
            C_ = int(name[6]) if rows else 0
            fits = not rows or (nx <= 64 * C_ and nx % C_ == 0)
            if not fits:
                assert st == rpr.RPR_ERR_UNSUPPORTED, name
                continue
            assert st == 0, (name, rpr.last_error())
            err = rel_err(host(xout), ref)
            print(nx, ny, name, "fp64" if prec == rpr.RPR_FP64 else "fp32", "rel err %.2e" % err)
            assert np.all(np.isfinite(host(xout))), name
            assert err <= (1e-12 if prec == rpr.RPR_FP64 else 2e-5), name
            served += 1
    finally:
        rpr.rpr_tune_set(key, -1)
    assert served >= 1


@pytest.mark.parametrize("steps", [1, 3])
@pytest.mark.parametrize("kind,nx,ny,params", [(rpr.RPR_BRUSS2D, 70, 37, (1.0, 3.0, 0.02, 0.01)),
                                               (rpr.RPR_DIFFREACT2D, 67, 17, (1e-3, 5e-3, 5e-3)),
                                               (rpr.RPR_SWE2D, 61, 45, (9.81,))],
                         ids=["bruss_70x37", "diffreact_67x17", "swe_61x45"])
@pytest.mark.parametrize("prec", [rpr.RPR_FP64, rpr.RPR_MIXED], ids=["fp64", "fp32"])
def test_tiled_rk4_single_and_odd_step_counts(orc, kind, nx, ny, params, steps, prec):
    """The one-pass RK4 tiles alternate the state between two work arrays:
    one step goes from the input straight to the output, an odd count ends
    on the other array than an even one."""
    rng = np.random.default_rng(steps + nx)
    d = rpr.nspecies(kind) * nx * ny
    X = np.stack([initial_state(kind, nx, ny, rng) for _ in range(2)])
    dom = (0, 1, 0, 1) if kind == rpr.RPR_SWE2D else (-1, 1, -1, 1)
    ref = orc.propagate_many(orc.problem(kind, nx, ny, dom, params), 4, steps, 2e-4, X)
    dtype = torch.float64 if prec == rpr.RPR_FP64 else torch.float32
    xin, xout = dev(X, dtype), torch.empty((2, d), dtype=dtype, device="cuda")
    rpr.rpr_propagate(rpr.make_rhs(kind, nx, ny, dom, params), d, 4, steps, prec, 2e-4, 2, xin, xout, threads=256)
    assert rel_err(host(xout), ref) <= (1e-12 if prec == rpr.RPR_FP64 else 2e-5)


def test_large_state_takes_the_tiled_form_automatically(orc):
    # 128 x 128 Brusselator in FP64 (256 KiB) does not fit one work-group
    kind, nx, ny, params = rpr.RPR_BRUSS2D, 128, 128, (1.0, 3.0, 0.02, 0.01)
    rng = np.random.default_rng(8)
    X = np.stack([initial_state(kind, nx, ny, rng) for _ in range(2)])
    ref = orc.propagate_many(orc.problem(kind, nx, ny, (-1, 1, -1, 1), params), 4, 10, 1e-4, X)
    xout = torch.empty((2, X.shape[1]), dtype=torch.float64, device="cuda")
    rpr.rpr_propagate(rpr.make_rhs(kind, nx, ny, params=params), X.shape[1], 4, 10, rpr.RPR_FP64, 1e-4, 2, dev(X),
                      xout)
    assert rel_err(host(xout), ref) <= 1e-12


def test_propagate_many_states_is_batched_identically(orc):
    # every state of a batch goes through the same kernel: equal inputs give bitwise equal outputs
    kind, nx, ny = rpr.RPR_DIFFREACT2D, 64, 64
    rng = np.random.default_rng(3)
    x = rng.standard_normal(2 * nx * ny)
    X = np.stack([x] * 5)
    xin, xout = dev(X), torch.empty((5, X.shape[1]), dtype=torch.float64, device="cuda")
    rpr.rpr_propagate(rpr.make_rhs(kind, nx, ny, params=(1e-3, 5e-3, 5e-3)), X.shape[1], 4, 50, rpr.RPR_FP64,
                      1e-4, 5, xin, xout)
    got = host(xout)
    for r in range(1, 5):
        np.testing.assert_array_equal(got[r], got[0])


def test_bruss_fixed_point_exact_on_gpu():
    nx = ny = 64
    u = np.concatenate([np.full(nx * ny, 1.0), np.full(nx * ny, 3.0)])[None]
    xin, xout = dev(u), torch.empty_like(dev(u))
    rpr.rpr_propagate(rpr.make_rhs(rpr.RPR_BRUSS2D, nx, ny, params=(1.0, 3.0, 0.02, 0.01)), u.shape[1], 4, 100,
                      rpr.RPR_FP64, 1e-3, 1, xin, xout)
    np.testing.assert_array_equal(host(xout), u)


@pytest.mark.parametrize("n,M,d,act", [(37, 50, 300, 0), (64, 200, 8192, 1), (5, 13, 1000, 0), (1, 3, 7, 1)])
def test_features_match_oracle(orc, n, M, d, act):
    rng = np.random.default_rng(n + M + d)
    A = rng.uniform(-1, 1, (M, d))
    zeta = rng.uniform(-1, 1, M)
    X = rng.standard_normal((n, d))
    s = 4.0
    ref = orc.features(orc.Net(A, zeta, act, 0.0, s), X)
    Phi = torch.empty((n, M), dtype=torch.float64, device="cuda")
    rpr.rpr_randnet_features(M, d, n, act, s, dev(A), dev(zeta), dev(X), Phi)
    err = rel_err(host(Phi), ref)
    print("features", n, M, d, "rel err %.2e" % err)
    assert err <= 1e-13


# M around the 32-column panel size of the factorisation (one block, ragged
# last block, several blocks, the largest M) and d around the 32-column
# blocks of the solve
@pytest.mark.parametrize("n,M,d", [(40, 30, 77), (12, 100, 128), (300, 200, 1000), (1, 5, 3), (50, 32, 32),
                                   (70, 33, 65), (90, 64, 31), (150, 97, 200), (600, 512, 300)])
def test_ridge_fit_matches_oracle(orc, n, M, d):
    rng = np.random.default_rng(n * M)
    Phi = np.tanh(rng.standard_normal((n, M)))
    Y = rng.standard_normal((n, d))
    lam = 1e-3
    ref = orc.ridge_fit(Phi, Y, lam)
    W = torch.empty((M, d), dtype=torch.float64, device="cuda")
    rpr.rpr_ridge_fit(M, d, n, dev(Phi), dev(Y), lam, W)
    kappa = np.linalg.cond(Phi.T @ Phi + lam * np.eye(M))
    tol = max(1e-12, 10 * kappa * 2.0 ** -53)
    err = rel_err(host(W), ref)
    print("ridge", n, M, d, "kappa %.1e rel err %.2e tol %.1e" % (kappa, err, tol))
    assert err <= tol


def test_ridge_fit_reports_non_positive_definite():
    # a NaN feature makes every pivot after it NaN: the factorisation fails
    # (reported, W zeroed) instead of returning garbage
    rng = np.random.default_rng(5)
    n, M, d = 20, 40, 50
    Phi = np.tanh(rng.standard_normal((n, M)))
    Phi[3, 7] = np.nan
    W = torch.full((M, d), 7.0, dtype=torch.float64, device="cuda")
    with pytest.raises(rpr.RprError) as e:
        rpr.rpr_ridge_fit(M, d, n, dev(Phi), dev(rng.standard_normal((n, d))), 1e-3, W)
    assert e.value.status == rpr.RPR_ERR_NOT_SPD
    assert np.all(host(W) == 0.0)


def test_readout_matches_oracle_formula():
    rng = np.random.default_rng(11)
    M, d, n = 30, 77, 9
    W = rng.standard_normal((M, d))
    Phi = rng.standard_normal((n, M))
    out = torch.empty((n, d), dtype=torch.float64, device="cuda")
    rpr.rpr_randnet_readout(M, d, n, dev(W), dev(Phi), out)
    assert rel_err(host(out), Phi @ W) <= 1e-13


def test_uniform_generator_bitwise(orc):
    for seed, first, n in [(0, 0, 1000), (12345, 7, 100003)]:
        out = torch.empty(n, dtype=torch.float64, device="cuda")
        rpr.rpr_uniform_pm1(seed, first, n, out)
        np.testing.assert_array_equal(host(out), orc.uniform_pm1(seed, first, n))


@pytest.mark.parametrize("n,M,d,act", [(64, 200, 8192, 1), (37, 50, 300, 0), (5, 13, 1000, 0), (130, 70, 96, 1),
                                       (8, 300, 110592, 1), (300, 200, 4096, 1), (256, 300, 2056, 0),
                                       (200, 150, 722, 0)])
def test_split_bf16_features_close_to_fp64_oracle(orc, n, M, d, act):
    """Split-bfloat16 features against the FP64 features of the same (FP32)
    inputs.  Per product the three-piece splits leave <= 2^-27 of each factor
    and the six kept products drop terms <= 3 2^-24 |a x|; the FP32 sums run
    over at most 6 x 2048 products per K split (d <= 131072).  Bound on the pre-activation
    (sigma is 1-Lipschitz): 2^-16 sum_j |a x_j / s|, about 8 x the summation
    error of a random walk over 12288 FP32 additions."""
    rng = np.random.default_rng(n * 7 + d)
    A = rng.uniform(-1, 1, (M, d))
    zeta = rng.uniform(-1, 1, M)
    X = rng.standard_normal((n, d)).astype(np.float32)
    s = 4.0
    ref = orc.features(orc.Net(A, zeta, act, 0.0, s), X.astype(np.float64))
    Phi = torch.empty((n, M), dtype=torch.float64, device="cuda")
    rpr.rpr_randnet_features_bf16(M, d, n, act, s, dev(A), dev(zeta), dev(X, torch.float32), Phi)
    got = host(Phi)
    S = np.abs(X.astype(np.float64) / s) @ np.abs(A).T
    ratio = np.abs(got - ref) / S
    print("split bf16 features", n, M, d, "max |diff| / sum|a x| = %.2e (bound %.2e)" % (ratio.max(), 2.0 ** -16))
    assert np.all(np.abs(got - ref) <= 2.0 ** -16 * S)


@pytest.mark.parametrize("n,M,d", [(300, 200, 4096), (130, 70, 96), (256, 300, 2056)])
def test_split_bf16_large_tiles_equal_small_tiles(n, M, d):
    # More than 16 rows with d % 8 == 0 take the 128 x 128-tile kernel on
    # inputs split beforehand; 16 rows take the 64 x 64-tile kernel that
    # splits on the fly.  A row's features do not depend on the other rows,
    # and both kernels use the same K split, K steps and product order: every
    # block of 16 rows of the large call must equal the small call on those
    # rows bit for bit.
    rng = np.random.default_rng(n + M + d)
    A = rng.uniform(-1, 1, (M, d))
    zeta = rng.uniform(-1, 1, M)
    X = rng.standard_normal((n, d)).astype(np.float32)
    Ad, zd = dev(A), dev(zeta)
    big = torch.empty((n, M), dtype=torch.float64, device="cuda")
    rpr.rpr_randnet_features_bf16(M, d, n, 1, 2.0, Ad, zd, dev(X, torch.float32), big)
    big = host(big)
    for r0 in range(0, n, 16):
        rows = X[r0:r0 + 16]
        small = torch.empty((rows.shape[0], M), dtype=torch.float64, device="cuda")
        rpr.rpr_randnet_features_bf16(M, d, rows.shape[0], 1, 2.0, Ad, zd, dev(rows, torch.float32), small)
        np.testing.assert_array_equal(big[r0:r0 + 16], host(small))
