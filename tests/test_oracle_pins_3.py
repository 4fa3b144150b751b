"""Pins of the oracle's eighth-order Runge-Kutta fine solver (Cooper and
Verner's 11-stage method; the paper's Burgers and diffusion-reaction runs
use an RK8 fine solver) and of its three-dimensional Brusselator (App. E):
the tableau against every order condition up to order 8 (rooted trees),
the integrator against the stability function on exact eigenvectors and
against its convergence order, the 3D system against its fixed point, its
Fourier modes, its symmetries and the 2D system.  No GPU needed."""
import itertools
import math
from functools import lru_cache

import numpy as np
import pytest


# ---- rooted trees and the order conditions of Butcher's theory ----
@lru_cache(maxsize=None)
def trees(n):
    """Rooted trees with n vertices, each a sorted tuple of its subtrees."""
    if n == 1:
        return [()]
    out = set()
    # partitions of n - 1 vertices into subtrees
    def parts(rem, maxsize):
        if rem == 0:
            yield []
            return
        for k in range(min(rem, maxsize), 0, -1):
            for rest in parts(rem - k, k):
                yield [k] + rest
    for p in parts(n - 1, n - 1):
        for combo in itertools.product(*[trees(k) for k in p]):
            out.add(tuple(sorted(combo)))
    return sorted(out)


def order_of(t):
    return 1 + sum(order_of(s) for s in t)


def gamma(t):
    return order_of(t) * math.prod(gamma(s) for s in t)


def stage_weights(t, A):
    """Vector g(t) with g(root alone) = 1 and g(t) = prod_k (A g(t_k))."""
    v = np.ones(A.shape[0])
    for s in t:
        v = v * (A @ stage_weights(s, A))
    return v


def test_tree_counts():
    # numbers of rooted trees of order 1..8 (OEIS A000081)
    assert [len(trees(n)) for n in range(1, 9)] == [1, 1, 2, 4, 9, 20, 48, 115]


def test_rk8_tableau_satisfies_every_order_condition_up_to_8(orc):
    A, b, c = orc.rk_tableau(8)
    assert A.shape == (11, 11) and np.allclose(np.triu(A), 0.0)
    np.testing.assert_allclose(A.sum(axis=1), c, rtol=0, atol=1e-15)
    worst = 0.0
    for n in range(1, 9):
        for t in trees(n):
            phi = b @ stage_weights(t, A)
            worst = max(worst, abs(phi - 1.0 / gamma(t)) * gamma(t))
    assert worst < 1e-12, worst
    # and it is not of order 9: some condition of order 9 fails
    miss = max(abs(b @ stage_weights(t, A) - 1.0 / gamma(t)) * gamma(t) for t in trees(9))
    assert miss > 1e-3


def test_rk4_tableau_satisfies_order_4_only(orc):
    A, b, c = orc.rk_tableau(4)
    for n in range(1, 5):
        for t in trees(n):
            assert abs(b @ stage_weights(t, A) - 1.0 / gamma(t)) < 1e-15
    assert max(abs(b @ stage_weights(t, A) - 1.0 / gamma(t)) for t in trees(5)) > 1e-3


def stability_function(A, b, z):
    s = len(b)
    return 1 + z * b @ np.linalg.solve(np.eye(s) - z * A, np.ones(s))


def mode3(n, kx, ky, kz):
    x = np.arange(n)
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")  # X: z index, Y: y index, Z: x index
    return np.cos(2 * np.pi * (kx * Z + ky * Y + kz * X) / n).ravel()


@pytest.mark.parametrize("method", [1, 4, 8])
def test_bruss3d_fourier_modes_decay_by_the_stability_function(orc, method):
    # A = B = 0, v = 0: u_t = Du lap u - u; a periodic Fourier mode of the
    # seven-point Laplacian has eigenvalue -(4/dx^2)(sin^2(pi kx/n) + sin^2(pi ky/n)
    # + sin^2(pi kz/n)), and one RK step multiplies it by R(mu dt), R the
    # method's stability function (from its tableau)
    n, Du, dt, steps = 8, 0.01, 0.01, 20
    pb = orc.problem(orc.BRUSS3D, n, n, params=(0.0, 0.0, Du, 0.02), nz=n)
    assert orc.dim(pb) == 2 * n ** 3
    A, b, _ = orc.rk_tableau(method)
    dx = 2.0 / n
    for kx, ky, kz in [(1, 0, 0), (1, 2, 3), (4, 4, 4)]:
        m = mode3(n, kx, ky, kz)
        lam = -(4 / dx ** 2) * (np.sin(np.pi * kx / n) ** 2 + np.sin(np.pi * ky / n) ** 2 +
                                np.sin(np.pi * kz / n) ** 2)
        amp = stability_function(A, b, (Du * lam - 1.0) * dt) ** steps
        out = orc.propagate(pb, method, steps, dt, np.concatenate([m, np.zeros(n ** 3)]))
        np.testing.assert_allclose(out[: n ** 3], amp * m, rtol=0, atol=1e-13 * max(1.0, abs(amp)))
        np.testing.assert_array_equal(out[n ** 3:], 0.0)


@pytest.mark.parametrize("method", [1, 4, 8])
def test_bruss3d_fixed_point_is_exact(orc, method):
    pb = orc.problem(orc.BRUSS3D, 5, 4, params=(1.0, 3.0, 0.1, 0.01), nz=3)
    u0 = np.concatenate([np.full(60, 1.0), np.full(60, 3.0)])
    np.testing.assert_array_equal(orc.propagate(pb, method, 7, 1e-3, u0), u0)


def test_bruss3d_axis_permutations_commute_with_the_right_hand_side(orc):
    # on a cubic grid of a cube, swapping the x and z axes (or x and y) of the
    # state swaps those axes of h(u) (up to the order in which the three
    # second differences are added: rounding)
    n = 6
    pb = orc.problem(orc.BRUSS3D, n, n, params=(1.0, 3.0, 0.1, 0.01), nz=n)
    rng = np.random.default_rng(4)
    u = np.concatenate([1 + 0.2 * rng.standard_normal(n ** 3), 3 + 0.2 * rng.standard_normal(n ** 3)])
    h = orc.rhs(pb, u).reshape(2, n, n, n)
    for axes in ((0, 2), (1, 2)):
        perm = [0, 1, 2, 3]
        perm[axes[0] + 1], perm[axes[1] + 1] = perm[axes[1] + 1], perm[axes[0] + 1]
        up = u.reshape(2, n, n, n).transpose(perm).ravel()
        np.testing.assert_allclose(orc.rhs(pb, up).reshape(2, n, n, n), h.transpose(perm), rtol=0,
                                   atol=1e-14 * np.abs(h).max())


def test_bruss3d_with_one_layer_is_the_2d_system(orc):
    # nz = 1: the z part of the seven-point Laplacian is (f - 2f + f)/dz^2 = 0
    nx, ny = 7, 5
    p3 = orc.problem(orc.BRUSS3D, nx, ny, params=(1.0, 3.0, 0.02, 0.01), nz=1)
    p2 = orc.problem(orc.BRUSS2D, nx, ny, params=(1.0, 3.0, 0.02, 0.01))
    rng = np.random.default_rng(5)
    u = np.concatenate([1 + 0.1 * rng.standard_normal(nx * ny), 3 + 0.1 * rng.standard_normal(nx * ny)])
    np.testing.assert_allclose(orc.rhs(p3, u), orc.rhs(p2, u), rtol=1e-15, atol=1e-15)


def test_rk8_converges_at_order_8(orc):
    # viscous Burgers on a coarse periodic grid, one slice of T = 0.5: halving
    # dt from 16 to 32 steps divides the error against a 40x finer RK8
    # solution by about 2^8 (measured 303: near the asymptotic regime), where
    # classical RK4 divides it by about 2^4
    d, nu, T = 16, 0.05, 0.5
    pb = orc.problem(orc.BURGERS1D, d, params=(nu,))
    x = -1 + 2 * np.arange(d) / d
    u0 = np.sin(np.pi * x) + 0.5 * np.cos(2 * np.pi * x)
    ref = orc.propagate(pb, 8, 1280, T / 1280, u0)
    errs = [np.abs(orc.propagate(pb, 8, n, T / n, u0) - ref).max() for n in (16, 32)]
    ratio = errs[0] / errs[1]
    assert errs[1] > 1e-13, errs  # above rounding
    assert 200 < ratio < 340, (errs, ratio)
    e4 = [np.abs(orc.propagate(pb, 4, n, T / n, u0) - ref).max() for n in (20, 40)]
    assert 12 < e4[0] / e4[1] < 21


def test_rk8_is_exact_on_polynomials_of_degree_8_in_time(orc):
    # Burgers with nu = 0 at a constant state is stationary; a quicker exact
    # check of the step: the linear heat equation's Fourier mode over one
    # step equals the degree-11 stability polynomial whose first 9 Taylor
    # coefficients are those of exp
    A, b, _ = orc.rk_tableau(8)
    coef = [1.0] + [b @ np.linalg.matrix_power(A, p - 1) @ np.ones(len(b)) for p in range(1, 12)]
    for p in range(0, 9):
        assert abs(coef[p] - 1 / math.factorial(p)) < 1e-14 / math.factorial(p) + 1e-16
    assert abs(coef[9] - 1 / math.factorial(9)) > 1e-7


def test_bruss3d_stability_bound_uses_the_seven_point_laplacian(orc):
    n, Du = 6, 0.05
    pb = orc.problem(orc.BRUSS3D, n, n, params=(0.0, 0.0, Du, 0.01), nz=n)
    u = np.zeros(2 * n ** 3)
    dx = 2.0 / n
    rho = Du * 12 / dx ** 2 + 1.0
    assert orc.stability(pb, 1, 0.01, u) == pytest.approx(0.01 * rho / 2, rel=1e-14)
    assert orc.stability(pb, 8, 0.01, u) == pytest.approx(0.01 * rho / 2.9, rel=1e-14)
    # the checkerboard mode decays just below the forward-Euler limit and grows above it
    m = mode3(n, n // 2, n // 2, n // 2)
    dt1 = 1.0 / orc.stability(pb, 1, 1.0, u)
    for frac, grows in ((0.99, False), (1.01, True)):
        out = orc.propagate(pb, 1, 300, frac * dt1, np.concatenate([m, np.zeros(n ** 3)]))
        assert (np.abs(out[: n ** 3]).max() > 1.0) == grows
    # RK8: the real-axis limit of its stability function lies beyond 2.9
    A, b, _ = orc.rk_tableau(8)
    assert abs(stability_function(A, b, -2.9)) < 1 and abs(stability_function(A, b, -3.8)) > 1
    assert abs(stability_function(A, b, 2.9j)) <= 1 + 1e-12
