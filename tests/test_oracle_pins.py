"""Pins of the CPU oracle to facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: closed-form
solutions of the discrete schemes, hand-computed values (tests/golden),
invariants the paper states, textbook convergence orders, or numpy/scipy
library routines.  No GPU is needed.
"""
import json
import math
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rk4_amp(z):
    return 1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24


# ---------------------------------------------------------------- generator --
def test_splitmix64_reference_outputs(orc):
    # First outputs of SplitMix64 (Steele, Lea & Flood, OOPSLA 2014) from state 0.
    assert orc.splitmix64(0, 0) == 0xE220A8397B1DCDAF
    assert orc.splitmix64(0, 1) == 0x6E789E6AA1B965F4
    assert orc.splitmix64(0, 2) == 0x06C45D188009454F


def test_uniform_pm1_range_and_moments(orc):
    x = orc.uniform_pm1(12345, 0, 200000)
    assert x.min() >= -1.0 and x.max() < 1.0
    assert abs(x.mean()) < 0.01 and abs(x.var() - 1 / 3) < 0.01
    # counter-based: any window reproduces the same stream
    np.testing.assert_array_equal(orc.uniform_pm1(12345, 1000, 10), x[1000:1010])


# ----------------------------------------------------------- right-hand sides --
def test_reaction_terms_at_constant_states(orc):
    g = json.load(open(os.path.join(GOLDEN, "reaction_constants.json")))
    for case in g["diffreact"]:
        pb = orc.problem(orc.DIFFREACT2D, 4, 3, params=(1e-3, 5e-3, case["c"]))
        u = np.concatenate([np.full(12, case["u"]), np.full(12, case["v"])])
        h = orc.rhs(pb, u)
        np.testing.assert_allclose(h[:12], case["hu"], rtol=1e-15, atol=1e-17)
        np.testing.assert_allclose(h[12:], case["hv"], rtol=1e-15, atol=1e-17)
    for case in g["bruss"]:
        pb = orc.problem(orc.BRUSS2D, 4, 3, params=(case["A"], case["B"], 0.02, 0.01))
        u = np.concatenate([np.full(12, case["u"]), np.full(12, case["v"])])
        h = orc.rhs(pb, u)
        np.testing.assert_array_equal(h[:12], case["hu"])
        np.testing.assert_array_equal(h[12:], case["hv"])


def test_bruss_fixed_point_is_exact(orc):
    # (u, v) = (A, B/A) is a steady state; with A = 1, B = 3 every term is exact.
    pb = orc.problem(orc.BRUSS2D, 8, 8, params=(1.0, 3.0, 0.02, 0.01))
    u0 = np.concatenate([np.full(64, 1.0), np.full(64, 3.0)])
    out = orc.propagate(pb, 4, 50, 1e-3, u0)
    np.testing.assert_array_equal(out, u0)


def periodic_mode(n, kx, ky):
    x = np.arange(n)
    return np.cos(2 * np.pi * (kx * x[None, :] + ky * x[:, None]) / n)


@pytest.mark.parametrize("method", [1, 4])
def test_bruss_linear_mode_decay_matches_closed_form(orc, method):
    # With A = B = 0 and v = 0: u_t = Du lap_h u - u, a linear system whose Fourier
    # modes are exact eigenvectors of the periodic 5-point Laplacian with
    # eigenvalue -(4/dx^2)(sin^2(pi kx/n) + sin^2(pi ky/n)); one RK step multiplies
    # a mode by the stability polynomial R(mu dt).
    n, Du, dt, steps = 16, 0.02, 2e-3, 40
    pb = orc.problem(orc.BRUSS2D, n, n, params=(0.0, 0.0, Du, 0.01))
    dx = 2.0 / n
    for kx, ky in [(1, 0), (2, 3), (5, 7)]:
        mode = periodic_mode(n, kx, ky).ravel()
        lam = -(4 / dx ** 2) * (np.sin(np.pi * kx / n) ** 2 + np.sin(np.pi * ky / n) ** 2)
        mu = Du * lam - 1.0
        z = mu * dt
        amp = (1 + z) ** steps if method == 1 else rk4_amp(z) ** steps
        u0 = np.concatenate([mode, np.zeros(n * n)])
        out = orc.propagate(pb, method, steps, dt, u0)
        np.testing.assert_allclose(out[: n * n], amp * mode, rtol=0, atol=1e-13 * abs(amp) + 1e-15)
        np.testing.assert_array_equal(out[n * n:], 0.0)
    # v alone: v_t = Dv lap_h v (u = 0 stays 0 because A = 0 and u^2 v = 0)
    Dv = 0.01
    mode = periodic_mode(n, 3, 1).ravel()
    lam = -(4 / dx ** 2) * (np.sin(np.pi * 3 / n) ** 2 + np.sin(np.pi * 1 / n) ** 2)
    z = Dv * lam * dt
    amp = (1 + z) ** steps if method == 1 else rk4_amp(z) ** steps
    out = orc.propagate(pb, method, steps, dt, np.concatenate([np.zeros(n * n), mode]))
    np.testing.assert_allclose(out[n * n:], amp * mode, rtol=0, atol=1e-13)


def neumann_mode(n, k):
    # DCT-II vector: exact eigenvector of the mirror-ghost second difference with
    # eigenvalue -(4/dx^2) sin^2(pi k / (2n)).
    return np.cos(np.pi * k * (np.arange(n) + 0.5) / n)


def test_diffreact_neumann_laplacian_eigenvectors(orc):
    nx, ny = 12, 9
    Du, Dv, c = 1e-3, 5e-3, 5e-3
    pb = orc.problem(orc.DIFFREACT2D, nx, ny, params=(Du, Dv, c))
    dx, dy = 2.0 / nx, 2.0 / ny
    for kx, ky in [(0, 1), (3, 2), (11, 8)]:
        mode = np.outer(neumann_mode(ny, ky), neumann_mode(nx, kx)).ravel()
        lam = -(4 / dx ** 2) * np.sin(np.pi * kx / (2 * nx)) ** 2 - (4 / dy ** 2) * np.sin(np.pi * ky / (2 * ny)) ** 2
        # v = mode, u = 0: h_v = Dv lap v + u - v = (Dv lam - 1) v, h_u = -c - v
        h = orc.rhs(pb, np.concatenate([np.zeros(nx * ny), mode]))
        np.testing.assert_allclose(h[nx * ny:], (Dv * lam - 1) * mode, rtol=0, atol=1e-13)
        np.testing.assert_allclose(h[: nx * ny], -c - mode, rtol=0, atol=1e-15)
        # u = eps * mode, v = 0: h_u + c = (Du lam + 1) eps mode + O(eps^3)
        eps = 1e-7
        h = orc.rhs(pb, np.concatenate([eps * mode, np.zeros(nx * ny)]))
        np.testing.assert_allclose((h[: nx * ny] + c) / eps, (Du * lam + 1) * mode, rtol=0, atol=1e-9)
        np.testing.assert_allclose(h[nx * ny:], eps * mode, rtol=1e-15, atol=0)


def test_burgers_diffusion_mode_small_amplitude(orc):
    d, nu = 64, 0.01
    pb = orc.problem(orc.BURGERS1D, d, params=(nu,))
    dx = 2.0 / d
    for k in (1, 5, 17):
        mode = np.sin(2 * np.pi * k * np.arange(d) / d)
        eps = 1e-9
        h = orc.rhs(pb, eps * mode) / eps
        lam = -(4 / dx ** 2) * np.sin(np.pi * k / d) ** 2
        # the advection term is O(eps) relative to the diffusion term
        np.testing.assert_allclose(h, nu * lam * mode, rtol=0, atol=1e-6 * abs(nu * lam) + 1e-12)


def test_burgers_rhs_sums_to_zero(orc):
    # Both the central second difference and u_j (u_{j+1} - u_{j-1}) telescope on
    # the periodic grid, so sum_j h_j = 0 and sum_j u_j is conserved.
    rng = np.random.default_rng(0)
    d = 128
    pb = orc.problem(orc.BURGERS1D, d, params=(0.01,))
    u = rng.normal(size=d)
    h = orc.rhs(pb, u)
    assert abs(h.sum()) <= 1e-13 * np.abs(h).sum()
    out = orc.propagate(pb, 4, 500, 1e-4, u)
    assert abs(out.sum() - u.sum()) <= 1e-12 * np.abs(u).sum()


def cole_hopf(x, t, nu, a, k, xc):
    # phi = 1 + a exp(-nu k^2 pi^2 t) cos(k pi (x - xc)) solves phi_t = nu phi_xx;
    # u = -2 nu phi_x / phi solves u_t + u u_x = nu u_xx (Cole-Hopf).
    e = a * np.exp(-nu * (k * np.pi) ** 2 * t)
    return 2 * nu * k * np.pi * e * np.sin(k * np.pi * (x - xc)) / (1 + e * np.cos(k * np.pi * (x - xc)))


def test_burgers_converges_to_cole_hopf_second_order(orc):
    nu, a, k, xc, T = 0.05, 0.8, 1, 0.3, 0.5
    errs = []
    for d in (32, 64, 128):
        x = -1 + 2 * np.arange(d) / d
        pb = orc.problem(orc.BURGERS1D, d, params=(nu,))
        steps = 4000
        out = orc.propagate(pb, 4, steps, T / steps, cole_hopf(x, 0.0, nu, a, k, xc))
        errs.append(np.abs(out - cole_hopf(x, T, nu, a, k, xc)).max())
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.4 < r1 < 4.6 and 3.4 < r2 < 4.6, errs
    assert errs[-1] < 2e-3


@pytest.mark.parametrize("method,order", [(1, 1), (4, 4)])
def test_time_refinement_order(orc, method, order):
    # Richardson ratio (u_n - u_2n) / (u_2n - u_4n) -> 2^order.
    d = 64
    pb = orc.problem(orc.BURGERS1D, d, params=(0.02,))
    x = -1 + 2 * np.arange(d) / d
    u0 = 0.5 * np.sin(np.pi * x) + 0.2 * np.cos(2 * np.pi * x)
    T = 0.2
    n = 200 if method == 1 else 25
    un, u2n, u4n = (orc.propagate(pb, method, m, T / m, u0) for m in (n, 2 * n, 4 * n))
    ratio = np.abs(un - u2n).max() / np.abs(u2n - u4n).max()
    assert abs(ratio / 2 ** order - 1) < 0.15, ratio


def test_swe_two_cell_hand_computed(orc):
    g = json.load(open(os.path.join(GOLDEN, "swe_two_cell.json")))
    p = g["problem"]
    pb = orc.problem(orc.SWE2D, p["nx"], p["ny"], domain=p["domain"], params=(p["g"],))
    np.testing.assert_array_equal(orc.rhs(pb, g["u"]), g["h"])


def test_swe_lake_at_rest_and_mass(orc):
    nx, ny = 24, 16
    pb = orc.problem(orc.SWE2D, nx, ny, domain=(0, 1, 0, 1), params=(9.81,))
    rest = np.concatenate([np.full(nx * ny, 1.3), np.zeros(2 * nx * ny)])
    np.testing.assert_array_equal(orc.propagate(pb, 4, 20, 1e-3, rest), rest)
    rng = np.random.default_rng(1)
    h = 1 + 0.1 * rng.random(nx * ny)
    q = np.concatenate([h, 0.05 * rng.normal(size=nx * ny), 0.05 * rng.normal(size=nx * ny)])
    out = orc.propagate(pb, 4, 100, 5e-4, q)
    assert abs(out[: nx * ny].sum() - h.sum()) <= 1e-13 * h.sum()


def test_swe_transpose_symmetry(orc):
    n = 20
    pb = orc.problem(orc.SWE2D, n, n, domain=(0, 1, 0, 1), params=(9.81,))
    rng = np.random.default_rng(2)
    h = 1 + 0.2 * rng.random((n, n))
    hu = 0.05 * rng.normal(size=(n, n))
    hv = 0.05 * rng.normal(size=(n, n))
    a = orc.propagate(pb, 4, 50, 5e-4, np.concatenate([h.ravel(), hu.ravel(), hv.ravel()]))
    b = orc.propagate(pb, 4, 50, 5e-4, np.concatenate([h.T.ravel(), hv.T.ravel(), hu.T.ravel()]))
    nc = n * n
    A = [a[s * nc:(s + 1) * nc].reshape(n, n) for s in range(3)]
    B = [b[s * nc:(s + 1) * nc].reshape(n, n) for s in range(3)]
    np.testing.assert_allclose(A[0], B[0].T, rtol=0, atol=1e-14)
    np.testing.assert_allclose(A[1], B[2].T, rtol=0, atol=1e-14)
    np.testing.assert_allclose(A[2], B[1].T, rtol=0, atol=1e-14)


def test_swe_standing_wave_speed(orc):
    # Small-amplitude standing wave h = 1 + eps cos(pi x) between walls at x = 0, 1:
    # linear theory gives h - 1 = eps cos(pi x) cos(pi sqrt(g h0) t); after half a
    # period the mode has flipped sign (Rusanov diffusion damps it by a few %).
    g, nx = 9.81, 256
    pb = orc.problem(orc.SWE2D, nx, 1, domain=(0, 1, 0, 1.0 / nx), params=(g,))
    xc = (np.arange(nx) + 0.5) / nx
    mode = np.cos(np.pi * xc)
    eps = 1e-3
    q0 = np.concatenate([1 + eps * mode, np.zeros(2 * nx)])
    T = 1 / math.sqrt(g)
    steps = 1000
    half = orc.propagate(pb, 4, steps, T / steps, q0)
    quarter = orc.propagate(pb, 4, steps // 2, T / steps, q0)
    c_half = (half[:nx] - 1) @ mode / (mode @ mode) / eps
    c_quarter = (quarter[:nx] - 1) @ mode / (mode @ mode) / eps
    assert -1.0 < c_half < -0.95, c_half
    assert abs(c_quarter) < 0.02, c_quarter


# ------------------------------------------------------------ random network --
def test_features_hand_example(orc):
    A = np.array([[1.0, -1.0], [0.5, 2.0]])
    zeta = np.array([0.25, -1.0])
    x = np.array([[1.0, 0.5]])  # x / s = (0.5, 0.25): z = (0.5, -0.25)
    relu = orc.features(orc.Net(A, zeta, orc.RELU, 0.0, 2.0), x)
    np.testing.assert_array_equal(relu, [[0.5, 0.0]])
    th = orc.features(orc.Net(A, zeta, orc.TANH, 0.0, 2.0), x)
    np.testing.assert_allclose(th, [[math.tanh(0.5), math.tanh(-0.25)]], rtol=1e-15)


def test_features_symmetries(orc):
    rng = np.random.default_rng(3)
    A = rng.uniform(-1, 1, (7, 5))
    X = rng.uniform(-1, 1, (4, 5))
    z0 = np.zeros(7)
    # tanh is odd: phi(-x) = -phi(x) when zeta = 0
    t = orc.Net(A, z0, orc.TANH, 0.0, 1.0)
    np.testing.assert_array_equal(orc.features(t, -X), -orc.features(t, X))
    # ReLU is positively homogeneous: phi(2x) = 2 phi(x) when zeta = 0
    r = orc.Net(A, z0, orc.RELU, 0.0, 1.0)
    np.testing.assert_array_equal(orc.features(r, 2 * X), 2 * orc.features(r, X))
    # scale: the network sees x / s
    r4 = orc.Net(A, z0, orc.RELU, 0.0, 4.0)
    np.testing.assert_array_equal(orc.features(r4, 4 * X), orc.features(r, X))


def svd_ridge(Phi, Y, lam):
    U, s, Vt = np.linalg.svd(Phi, full_matrices=False)
    return Vt.T @ np.diag(s / (s ** 2 + lam)) @ U.T @ Y


@pytest.mark.parametrize("n,M,d", [(12, 8, 3), (5, 8, 2), (8, 8, 1), (1, 4, 2)])
def test_ridge_primal_dual_svd_agree(orc, n, M, d):
    rng = np.random.default_rng(n * 100 + M)
    Phi = rng.normal(size=(n, M))
    Y = rng.normal(size=(n, d))
    lam = 1e-3
    ref = svd_ridge(Phi, Y, lam)
    Wp = orc.ridge_fit(Phi, Y, lam)
    Wd = orc.ridge_fit_dual(Phi, Y, lam)
    scale = np.abs(ref).max()
    # backward-stable solves: error <= O(kappa * unit roundoff) relative
    kp = np.linalg.cond(Phi.T @ Phi + lam * np.eye(M))
    kd = np.linalg.cond(Phi @ Phi.T + lam * np.eye(n))
    np.testing.assert_allclose(Wp, ref, rtol=0, atol=max(1e-12, 10 * kp * 2.0 ** -53) * scale)
    np.testing.assert_allclose(Wd, ref, rtol=0, atol=max(1e-12, 10 * kd * 2.0 ** -53) * scale)


def test_ridge_single_row_hand_formula(orc):
    # n = 1: W = phi (phi^T phi + lam)^{-1} y^T, so fhat(x_1) = |phi|^2/(|phi|^2 + lam) y.
    phi = np.array([[0.5, -0.25, 1.0]])
    y = np.array([[2.0, -1.0]])
    lam = 0.125
    W = orc.ridge_fit(phi, y, lam)
    n2 = float((phi @ phi.T)[0, 0])
    np.testing.assert_allclose(phi @ W, n2 / (n2 + lam) * y, rtol=1e-15)
    np.testing.assert_allclose(W, phi.T @ y / (n2 + lam), rtol=1e-15)


def test_ridgeless_limits(orc):
    rng = np.random.default_rng(5)
    # n < M: the lambda -> 0 limit is the min-norm interpolator pinv(Phi) Y (Sec. 4)
    # (dual form: well conditioned; primal form: error lambda/sigma_min^2 plus
    # kappa(Phi^T Phi + lambda I) times the unit roundoff)
    Phi = rng.normal(size=(4, 10))
    Y = rng.normal(size=(4, 3))
    ref = np.linalg.pinv(Phi) @ Y
    smin = np.linalg.svd(Phi, compute_uv=False).min()
    Wd = orc.ridge_fit_dual(Phi, Y, 1e-12)
    np.testing.assert_allclose(Wd, ref, rtol=0, atol=1e-10)
    np.testing.assert_allclose(Phi @ Wd, Y, rtol=0, atol=1e-10)
    lam = 1e-8
    kp = np.linalg.cond(Phi.T @ Phi + lam * np.eye(10))
    Wp = orc.ridge_fit(Phi, Y, lam)
    tol = (lam / smin ** 2 + 10 * kp * 2.0 ** -53) * np.abs(ref).max()
    np.testing.assert_allclose(Wp, ref, rtol=0, atol=tol)
    # n > M, full column rank: the limit is ordinary least squares
    Phi = rng.normal(size=(30, 6))
    Y = rng.normal(size=(30, 2))
    W = orc.ridge_fit(Phi, Y, 1e-12)
    np.testing.assert_allclose(W, np.linalg.lstsq(Phi, Y, rcond=None)[0], rtol=0, atol=1e-10)


def test_cholesky_against_numpy_and_failure(orc):
    rng = np.random.default_rng(6)
    X = rng.normal(size=(9, 9))
    S = X @ X.T + 0.1 * np.eye(9)
    np.testing.assert_allclose(orc.cholesky(S), np.linalg.cholesky(S), rtol=0, atol=1e-13)
    with pytest.raises(np.linalg.LinAlgError):
        orc.cholesky(-S)


def test_nearest_matches_stable_sort(orc):
    rng = np.random.default_rng(7)
    P = rng.integers(0, 3, size=(40, 3)).astype(float)  # many exact ties
    q = np.array([1.0, 1.0, 1.0])
    dist = ((P - q) ** 2).sum(1)
    for m in (1, 4, 11, 40):
        np.testing.assert_array_equal(orc.nearest(P, q, m), np.argsort(dist, kind="stable")[:m])


# ------------------------------------------------------------------- driver --
def burgers_case(orc, d=32, N=8, G_steps=20, F_steps=200, M=24, act=0, lam=1e-6, seed=0):
    rng = np.random.default_rng(seed)
    x = -1 + 2 * np.arange(d) / d
    a = rng.normal(0, 0.5, 4)
    u0 = sum(a[k - 1] * np.sin(k * np.pi * x) for k in range(1, 5))
    pb = orc.problem(orc.BURGERS1D, d, params=(0.02,))
    wr = np.random.default_rng(100 + seed)
    net = orc.Net(wr.uniform(-1, 1, (M, d)), wr.uniform(-1, 1, M), act, lam, 0.0)
    kw = dict(N=N, t0=0.0, tN=2.0, F=(4, F_steps), G=(1, G_steps))
    return pb, u0, net, kw


def test_eps_zero_gives_serial_fine_after_N(orc):
    pb, u0, net, kw = burgers_case(orc)
    N = kw["N"]
    U, info = orc.parareal(pb, u0, eps=0.0, net=net, keep_iterates=True, **kw)
    Uf = orc.serial_fine(pb, 4, kw["F"][1], (kw["tN"] / N) / kw["F"][1], N, u0)
    assert info["K"] == N and info["converged"]
    np.testing.assert_array_equal(info["L_hist"], np.arange(N + 1))
    np.testing.assert_array_equal(U, Uf)
    # after iteration k the first k slots hold the serial fine values exactly
    for k in range(1, N + 1):
        np.testing.assert_array_equal(info["U_iter"][k][: k + 1], Uf[: k + 1])


def test_eps_infinite_stops_after_one_iteration(orc):
    pb, u0, net, kw = burgers_case(orc)
    U, info = orc.parareal(pb, u0, eps=np.inf, net=net, **kw)
    assert info["K"] == 1 and info["L_final"] == kw["N"]


def test_frozen_prefix_and_L_monotone(orc):
    pb, u0, net, kw = burgers_case(orc, N=10)
    U, info = orc.parareal(pb, u0, eps=1e-7, net=net, keep_iterates=True, **kw)
    L = info["L_hist"]
    assert np.all(np.diff(L) >= 1)
    for k in range(1, info["K"] + 1):
        np.testing.assert_array_equal(info["U_iter"][k][: L[k - 1] + 1], info["U_iter"][k - 1][: L[k - 1] + 1])


@pytest.mark.parametrize("corr", [1, 0])
def test_G_equal_F_converges_in_one_iteration(orc, corr):
    # With G = F the coarse sweep is the serial fine solution and F - G = 0, so
    # both the classical and the RandNet corrections vanish.
    pb, u0, net, kw = burgers_case(orc)
    kw["G"] = kw["F"]
    U, info = orc.parareal(pb, u0, eps=1e-12, corr=corr, net=net, **kw)
    Uf = orc.serial_fine(pb, 4, kw["F"][1], (kw["tN"] / kw["N"]) / kw["F"][1], kw["N"], u0)
    assert info["K"] == 1
    np.testing.assert_array_equal(U, Uf)


def test_unstable_coarse_solver_still_reaches_serial_fine(orc):
    # Forward Euler far outside its stability region: every prediction is
    # non-finite, the pairs are dropped, and the exact-slot rule alone takes the
    # run to K = N with the serial fine result.
    pb, u0, net, kw = burgers_case(orc, d=64, G_steps=1)
    U, info = orc.parareal(pb, u0, eps=1e-6, net=net, **kw)
    Uf = orc.serial_fine(pb, 4, kw["F"][1], (kw["tN"] / kw["N"]) / kw["F"][1], kw["N"], u0)
    assert info["K"] == kw["N"] and info["nonfinite_rows"] > 0
    np.testing.assert_array_equal(U, Uf)


def test_first_iteration_uses_ridge_on_coarse_pairs(orc):
    # Iteration 1: pairs (U_{i-1}^0, F(U_{i-1}^0) - G(U_{i-1}^0)), i = 1..N, readout
    # from eq. "ridgeless", then U_2^1 = G(U_1^1) + W^T phi(U_1^1) with U_1^1 = F(u0).
    pb, u0, net, kw = burgers_case(orc)
    N = kw["N"]
    T = kw["tN"] / N
    U, info = orc.parareal(pb, u0, eps=1e-9, net=net, k_max=1, keep_iterates=True, **kw)
    U0 = info["U_iter"][0]
    Fv = orc.propagate_many(pb, 4, kw["F"][1], T / kw["F"][1], U0[:N])
    Gv = orc.propagate_many(pb, 1, kw["G"][1], T / kw["G"][1], U0[:N])
    s = 2.0 ** math.ceil(math.log2(max(1.0, np.abs(u0).max())))
    net_s = orc.Net(net.A, net.zeta, 0, 1e-6, s)
    Phi = orc.features(net_s, U0[:N])
    Wsvd = svd_ridge(Phi, Fv - Gv, 1e-6)
    x = U[1]
    np.testing.assert_array_equal(x, Fv[0])
    pred = orc.propagate(pb, 1, kw["G"][1], T / kw["G"][1], x) + (orc.features(net_s, x[None]) @ Wsvd)[0]
    np.testing.assert_allclose(U[2], pred, rtol=0, atol=1e-8 * np.abs(U[2]).max())


def test_nn_mode_with_all_rows_equals_global_fit(orc):
    # With m at least the number of stored pairs, the nearest-neighbour refit of
    # eq. "randnet" uses every pair, i.e. the same ridge estimator as the global
    # fit (dual versus primal form).
    pb, u0, net, kw = burgers_case(orc, lam=1e-3)
    a, ia = orc.parareal(pb, u0, eps=1e-8, net=net, k_max=2, corr=0, **kw)
    b, ib = orc.parareal(pb, u0, eps=1e-8, net=net, k_max=2, corr=2, m_nn=1000, **kw)
    assert ia["L_hist"].tolist() == ib["L_hist"].tolist()
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-9 * np.abs(a).max())
