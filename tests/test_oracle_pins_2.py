"""More pins of the CPU oracle: the classical correction of eq. "fpara"
against a closed-form scalar recursion, the default input scale on hand
values, and the stability bound of the propagators against assembled
Jacobians and against the growth of the discrete solution.  No GPU needed."""
import math

import numpy as np
import pytest


def rk4_amp(z):
    return 1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24


def periodic_mode(n, kx, ky):
    x = np.arange(n)
    return np.cos(2 * np.pi * (kx * x[None, :] + ky * x[:, None]) / n)


# ------------------------------------------------- classical Parareal, eq. "fpara" --
@pytest.mark.parametrize("G_steps", [1, 3])
def test_classical_parareal_iterates_follow_scalar_recursion(orc, G_steps):
    # Brusselator with A = B = 0 and v = 0 is the linear system u_t = Du lap_h u - u;
    # a periodic Fourier mode is an exact eigenvector (eigenvalue mu), so F and G
    # act on its amplitude as the scalars f = R4(mu dtF)^nF and g = (1 + mu dtG)^nG.
    # Classical Parareal (eq. "update_rule_generic" with the correction of eq.
    # "fpara", G evaluated at the previous iterate) then follows
    #   a_i^k = g a_{i-1}^k + (f - g) a_{i-1}^{k-1},
    # with a_i^0 = g^i, a_0^k = 1, and with eps = 0 the slots i <= k frozen at
    # iteration k after the exact slot a_k^k = f a_{k-1}^{k-1}.  Using G at the new
    # iterate instead (U_i = F(U_{i-1}^{k-1})) or dropping either term breaks it.
    # Du = 0.01 keeps G inside forward Euler's stability region for every mode
    # (dt rho = 0.25 * (0.01 * 512 + 1) = 1.5 with one step), so rounding in the
    # other modes is not amplified from slot to slot
    n, Du, N, tN, nF = 16, 0.01, 8, 2.0, 20
    pb = orc.problem(orc.BRUSS2D, n, n, params=(0.0, 0.0, Du, 0.05))
    dx = 2.0 / n
    mode = periodic_mode(n, 1, 2).ravel()
    lam = -(4 / dx ** 2) * (np.sin(np.pi * 1 / n) ** 2 + np.sin(np.pi * 2 / n) ** 2)
    mu = Du * lam - 1.0
    T = tN / N
    f = rk4_amp(mu * T / nF) ** nF
    g = (1 + mu * T / G_steps) ** G_steps
    assert abs(f - g) > 0.01  # the correction matters
    u0 = np.concatenate([mode, np.zeros(n * n)])
    U, info = orc.parareal(pb, u0, N=N, t0=0.0, tN=tN, F=(4, nF), G=(1, G_steps), eps=0.0, corr=orc.CORR_PARAREAL,
                           keep_iterates=True)
    assert info["K"] == N and info["L_hist"].tolist() == list(range(N + 1))
    a = np.zeros((N + 1, N + 1))
    a[0] = [g ** i for i in range(N + 1)]
    for k in range(1, N + 1):
        a[k, 0] = 1.0
        a[k, 1:k] = a[k - 1, 1:k]
        a[k, k] = f * a[k - 1, k - 1]
        for i in range(k + 1, N + 1):
            a[k, i] = g * a[k, i - 1] + (f - g) * a[k - 1, i - 1]
    # rounding only (a wrong correction moves values by ~|f - g| >= 0.01)
    Ui = info["U_iter"]
    for k in range(N + 1):
        for i in range(N + 1):
            np.testing.assert_allclose(Ui[k, i, : n * n], a[k, i] * mode, rtol=0, atol=1e-13)
            np.testing.assert_array_equal(Ui[k, i, n * n:], 0.0)
    # the fixed point is the serial fine solution f^i
    np.testing.assert_allclose(a[N], [f ** i for i in range(N + 1)], rtol=1e-13)


# ----------------------------------------------------------------- input scale --
@pytest.mark.parametrize("umax,s", [(0.0, 1.0), (0.5, 1.0), (1.0, 1.0), (1.5, 2.0), (2.0, 2.0), (3.0, 4.0),
                                    (4.0, 4.0), (4.000001, 8.0), (1000.0, 1024.0), (2.0 ** -3, 1.0)])
def test_input_scale_hand_values(orc, umax, s):
    # "Rescale so each coordinate lies in [-1, 1]": the smallest power of two
    # s >= max(1, ||u0||_inf); the sign of the extreme entry does not matter
    u = np.array([0.25, -umax, 0.1 * umax])
    assert orc.input_scale(u) == s
    assert orc.input_scale(-u) == s


# ------------------------------------------------------------- stability bound --
def jacobian(orc, pb, u, delta=1e-6):
    """Jacobian of the oracle's h at u by central differences."""
    d = u.size
    J = np.empty((d, d))
    for j in range(d):
        e = np.zeros(d)
        e[j] = delta
        J[:, j] = (orc.rhs(pb, u + e) - orc.rhs(pb, u - e)) / (2 * delta)
    return J


def test_stability_bound_is_the_spectral_radius_of_the_heat_operator(orc):
    # A = B = 0 at u = v = 0: J = diag(Du lap - 1, Dv lap); with Du >= Dv and an
    # even grid the largest |eigenvalue| is Du (4/dx^2 + 4/dy^2) + 1, which is
    # the bound (B + 1 = 1): dt / dt_max = dt rho / 2 for forward Euler
    n, Du = 8, 0.05
    pb = orc.problem(orc.BRUSS2D, n, n, params=(0.0, 0.0, Du, 0.01))
    u = np.zeros(2 * n * n)
    ev = np.linalg.eigvals(jacobian(orc, pb, u))
    rho = np.abs(ev).max()
    dx = 2.0 / n
    assert rho == pytest.approx(Du * 8 / dx ** 2 + 1, rel=1e-9)
    assert orc.stability(pb, 1, 0.01, u) == pytest.approx(0.01 * rho / 2, rel=1e-9)
    assert orc.stability(pb, 4, 0.01, u) == pytest.approx(0.01 * rho / 2.78, rel=1e-9)


@pytest.mark.parametrize("method,below,above", [(1, 0.99, 1.01), (4, 1.0, 1.01)])
def test_stability_limit_separates_decay_from_growth(orc, method, below, above):
    # the checkerboard mode (kx = ky = n/2) of the heat operator has the largest
    # |eigenvalue|; at dt / dt_max just below 1 it decays, just above it grows
    n, Du = 8, 0.05
    pb = orc.problem(orc.BRUSS2D, n, n, params=(0.0, 0.0, Du, 0.01))
    mode = periodic_mode(n, n // 2, n // 2).ravel()
    u0 = np.concatenate([mode, np.zeros(n * n)])
    dt1 = 1.0 / orc.stability(pb, method, 1.0, np.zeros(2 * n * n))  # dt_max
    for frac, grows in ((below, False), (above, True)):
        out = orc.propagate(pb, method, 400, frac * dt1, u0)
        amp = np.abs(out[: n * n]).max()
        assert (amp > 1.0) == grows, (method, frac, amp)


@pytest.mark.parametrize("U", [0.5, 1.5])
def test_forward_euler_condition_is_exact_for_burgers_at_a_constant_state(orc, U):
    # at u = U the Jacobian is nu D2 - U D1 (central), eigenvalues
    # -(2 nu/dx^2)(1 - cos t) - i (U/dx) sin t; forward Euler is stable iff
    # dt <= min(2 / rho_r, rho_r / (2 rho_i^2)) = min(dx^2/(2 nu), 2 nu / U^2)
    d, nu = 48, 0.02
    pb = orc.problem(orc.BURGERS1D, d, params=(nu,))
    u = np.full(d, U)
    ev = np.linalg.eigvals(jacobian(orc, pb, u))
    dx = 2.0 / d
    dt_max = min(dx ** 2 / (2 * nu), 2 * nu / U ** 2)
    assert orc.stability(pb, 1, dt_max, u) == pytest.approx(1.0, rel=1e-12)
    amp = lambda dt: np.abs(1 + dt * ev).max()
    assert amp(0.999 * dt_max) <= 1 + 1e-9
    assert amp(1.02 * dt_max) > 1 + 1e-9
    assert np.abs(ev.imag).max() <= U / dx * (1 + 1e-9)


@pytest.mark.parametrize("kind", ["diffreact", "bruss", "swe", "burgers"])
def test_stability_bound_covers_assembled_jacobians(orc, kind):
    # at random states the bound rho_r (+ rho_i) covers every eigenvalue of the
    # assembled Jacobian, so dt = dt_max keeps forward Euler's |1 + dt lam| <= 1
    # for the dissipative systems (all eigenvalues in the left half plane disc)
    rng = np.random.default_rng(7)
    if kind == "diffreact":
        pb = orc.problem(orc.DIFFREACT2D, 6, 5, params=(1e-2, 5e-2, 5e-3))
        u = rng.uniform(-1.5, 1.5, 60)
    elif kind == "bruss":
        pb = orc.problem(orc.BRUSS2D, 6, 6, params=(1.0, 3.0, 0.02, 0.01))
        u = np.concatenate([1 + 0.3 * rng.uniform(-1, 1, 36), 3 + 0.3 * rng.uniform(-1, 1, 36)])
    elif kind == "swe":
        pb = orc.problem(orc.SWE2D, 6, 5, domain=(0.0, 1.0, 0.0, 1.0), params=(9.81,))
        u = np.concatenate([1 + 0.2 * rng.uniform(0, 1, 30), 0.1 * rng.uniform(-1, 1, 60)])
    else:
        pb = orc.problem(orc.BURGERS1D, 32, params=(0.05,))
        u = rng.uniform(-1, 1, 32)
    ev = np.linalg.eigvals(jacobian(orc, pb, u))
    r1 = orc.stability(pb, 1, 1.0, u)   # = 1 / dt_max (forward Euler)
    r4 = orc.stability(pb, 4, 1.0, u)   # = (rho_r + rho_i) / 2.78
    assert np.abs(ev).max() <= 2.78 * r4 * (1 + 1e-7)
    if kind == "swe":
        # lake at rest: the Rusanov operator's eigenvalues lie in the disc about
        # -rho/2 of radius rho/2, so forward Euler at dt_max is stable
        ur = np.concatenate([np.full(30, 1.1), np.zeros(60)])
        evr = np.linalg.eigvals(jacobian(orc, pb, ur))
        assert np.abs(1 + evr / orc.stability(pb, 1, 1.0, ur)).max() <= 1 + 1e-7


def test_library_stability_matches_oracle(orc):
    # the library's host-side pre-check and the oracle's are written
    # separately; they agree on every system and method
    import paper_2411_06225_amd as rpr
    rng = np.random.default_rng(3)
    cases = [
        (rpr.RPR_BURGERS1D, 128, 1, (-1, 1, -1, 1), (0.01,), rng.normal(0, 0.5, 128)),
        (rpr.RPR_DIFFREACT2D, 16, 12, (-1, 1, -1, 1), (1e-3, 5e-3, 5e-3), rng.standard_normal(2 * 192)),
        (rpr.RPR_BRUSS2D, 16, 16, (-1, 1, -1, 1), (1.0, 3.0, 0.02, 0.01), 2 + rng.uniform(-1, 1, 512)),
        (rpr.RPR_SWE2D, 12, 10, (0, 1, 0, 1), (9.81,),
         np.concatenate([1 + rng.uniform(0, 0.2, 120), rng.uniform(-0.1, 0.1, 240)])),
    ]
    for kind, nx, ny, dom, par, u in cases:
        h = rpr.make_rhs(kind, nx, ny, dom, par)
        pb = orc.problem(kind, nx, ny, dom, par)
        speed = 0.0
        if kind == rpr.RPR_SWE2D:
            nc = nx * ny
            hh = u[:nc]
            speed = float((np.maximum(np.abs(u[nc:2 * nc]), np.abs(u[2 * nc:])) / hh + np.sqrt(9.81 * hh)).max())
        for method in (1, 4):
            for dt in (1e-4, 3e-3, 0.05):
                lib = rpr.rpr_stability(h, u.size, method, 1, dt, float(np.abs(u).max()), speed)
                assert lib == pytest.approx(orc.stability(pb, method, dt, u), rel=1e-13), (kind, method, dt)
