"""Pins of the oracle's ridgeless readout, the limit lambda -> 0 of eq.
"ridgeless" that Alg. "RandNets training procedure" writes as a
least-squares solve when the Gram has full rank and as a pseudo-inverse
otherwise: the cyclic Jacobi eigensolver under it, the least-squares and the
interpolation regimes against closed forms and library routines, a
rank-deficient case with a closed-form fit, and the driver's lambda = 0
branch as the limit of its pinned lambda > 0 branch.  No GPU needed."""
import numpy as np
import pytest


# ------------------------------------------------------------ eigensolver --
def test_sym_eig_two_by_two_closed_form(orc):
    a, b, c = 3.0, -1.25, 0.5
    w, V = orc.sym_eig(np.array([[a, b], [b, c]]))
    mid, rad = (a + c) / 2, np.hypot((a - c) / 2, b)
    np.testing.assert_allclose(np.sort(w), [mid - rad, mid + rad], rtol=1e-15, atol=1e-15)
    np.testing.assert_allclose(V.T @ V, np.eye(2), atol=1e-15)


@pytest.mark.parametrize("s", [1, 5, 17])
def test_sym_eig_reconstructs_and_matches_library(orc, s):
    rng = np.random.default_rng(s)
    B = rng.standard_normal((s, s))
    S = B + B.T
    w, V = orc.sym_eig(S)
    np.testing.assert_allclose(V.T @ V, np.eye(s), atol=1e-13)
    np.testing.assert_allclose(V @ np.diag(w) @ V.T, S, atol=1e-12 * np.abs(S).max())
    np.testing.assert_allclose(np.sort(w), np.linalg.eigvalsh(S), atol=1e-12 * np.abs(S).max())


def test_sym_eig_of_diagonal_is_identity_rotation(orc):
    S = np.diag([4.0, -1.0, 0.0, 2.5])
    w, V = orc.sym_eig(S)
    np.testing.assert_array_equal(w, np.diag(S))
    np.testing.assert_array_equal(V, np.eye(4))


# ------------------------------------------------------- ridgeless readout --
def test_full_rank_tall_is_least_squares(orc):
    # rank(X^T X) = M <= n: the least-squares estimator of the algorithm
    rng = np.random.default_rng(1)
    n, M, d = 40, 10, 3
    X, Y = rng.standard_normal((n, M)), rng.standard_normal((n, d))
    W, rank = orc.ridgeless_fit(X, Y)
    ref = np.linalg.lstsq(X, Y, rcond=None)[0]
    assert rank == M
    np.testing.assert_allclose(W, ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def test_wide_interpolates_with_minimum_norm(orc):
    # M >> n (Sec. 4, m nearest pairs and many neurons): the ridgeless
    # estimator interpolates the training data, with the least-norm weights
    rng = np.random.default_rng(2)
    n, M, d = 5, 60, 4
    X, Y = rng.standard_normal((n, M)), rng.standard_normal((n, d))
    W, rank = orc.ridgeless_fit(X, Y)
    assert rank == n
    np.testing.assert_allclose(X @ W, Y, atol=1e-12 * np.abs(Y).max())
    np.testing.assert_allclose(W, np.linalg.pinv(X) @ Y, atol=1e-12)
    # least norm: W lies in the row space of X
    P = X.T @ np.linalg.solve(X @ X.T, X)
    np.testing.assert_allclose(P @ W, W, atol=1e-12)


def test_duplicated_row_fits_the_mean_of_its_targets(orc):
    # two equal feature rows with targets y0 and y1: the least-squares fit at
    # that row is (y0 + y1) / 2; the other rows are still interpolated
    rng = np.random.default_rng(3)
    n, M, d = 6, 30, 2
    X, Y = rng.standard_normal((n, M)), rng.standard_normal((n, d))
    X[1] = X[0]
    W, rank = orc.ridgeless_fit(X, Y)
    assert rank == n - 1
    fit = X @ W
    np.testing.assert_allclose(fit[0], (Y[0] + Y[1]) / 2, atol=1e-11)
    np.testing.assert_allclose(fit[1], (Y[0] + Y[1]) / 2, atol=1e-11)
    np.testing.assert_allclose(fit[2:], Y[2:], atol=1e-11)


def test_rank_deficient_tall_matches_pseudo_inverse(orc):
    # n >= M but rank(X^T X) < M (two equal neurons): the pseudo-inverse branch
    rng = np.random.default_rng(4)
    n, M, d = 25, 8, 3
    X, Y = rng.standard_normal((n, M)), rng.standard_normal((n, d))
    X[:, 5] = X[:, 2]
    W, rank = orc.ridgeless_fit(X, Y)
    assert rank == M - 1
    np.testing.assert_allclose(W, np.linalg.pinv(X) @ Y, atol=1e-11)
    np.testing.assert_allclose(W[5], W[2], atol=1e-11)  # the least-norm split of equal neurons


def test_zero_features_give_zero_weights(orc):
    # ReLU features all switched off: the Gram is zero and so is the readout
    W, rank = orc.ridgeless_fit(np.zeros((4, 7)), np.ones((4, 2)))
    assert rank == 0
    np.testing.assert_array_equal(W, 0.0)


@pytest.mark.parametrize("n,M", [(30, 6), (4, 20)])
def test_ridge_approaches_the_ridgeless_limit(orc, n, M):
    # eq. "ridgeless" is the limit lambda -> 0 of the pinned ridge estimator;
    # lambda = 0 in ridge_fit / ridge_fit_dual takes the limit itself
    rng = np.random.default_rng(n + M)
    X, Y = rng.standard_normal((n, M)), rng.standard_normal((n, 2))
    W0, _ = orc.ridgeless_fit(X, Y)
    fit = orc.ridge_fit if n >= M else orc.ridge_fit_dual
    errs = [np.abs(fit(X, Y, lam) - W0).max() for lam in (1e-4, 1e-6, 1e-8)]
    assert errs[0] > errs[1] > errs[2] and errs[2] < 1e-6
    np.testing.assert_array_equal(orc.ridge_fit(X, Y, 0.0), W0)
    np.testing.assert_array_equal(orc.ridge_fit_dual(X, Y, 0.0), W0)


@pytest.mark.parametrize("n,M", [(30, 6), (5, 12)])
def test_from_statistics_equals_from_rows(orc, n, M):
    # the driver's global fit accumulates G = X^T X and B = X^T Y
    rng = np.random.default_rng(7 * n + M)
    X, Y = rng.standard_normal((n, M)), rng.standard_normal((n, 3))
    Ws, rs = orc.ridgeless_stats(X.T @ X, X.T @ Y, n)
    Wr, rr = orc.ridgeless_fit(X, Y)
    assert rs == rr == min(n, M)
    np.testing.assert_allclose(Ws, np.linalg.pinv(X) @ Y, atol=1e-9)
    np.testing.assert_allclose(Ws, Wr, atol=1e-9)


def test_nearest_pair_refit_reproduces_a_stored_pair(orc):
    # Sec. 4: with M >> m the refit interpolates its m pairs, so a query equal
    # to a stored input gets that pair's discrepancy back
    rng = np.random.default_rng(9)
    d, M, n, m = 12, 80, 20, 4
    P, Yp = rng.standard_normal((n, d)), rng.standard_normal((n, d))
    net = orc.Net(rng.uniform(-1, 1, (M, d)), rng.uniform(-1, 1, M), orc.RELU, 0.0, 4.0)
    q = P[13]
    idx = np.argsort(((P - q) ** 2).sum(1), kind="stable")[:m]
    W, rank = orc.ridgeless_fit(orc.features(net, P[idx]), Yp[idx])
    assert rank == m
    np.testing.assert_allclose(orc.features(net, q[None]) @ W, Yp[13][None], atol=1e-10)


# ---------------------------------------------------- the driver at lambda = 0 --
@pytest.mark.parametrize("corr", [0, 2], ids=["global", "nn"])
def test_driver_lambda_zero_is_the_limit_of_its_ridge_branch(orc, corr):
    # Burgers, few neurons (global: more pairs than neurons after the first
    # iteration, so the Gram has full rank and the ridge solution converges to
    # the ridgeless one as lambda -> 0); with eps = 0 every run takes k_max
    # iterations, and every iterate of the lambda = 0 run is approached by the
    # lambda > 0 runs
    nx, N = 32, 8
    pb = orc.problem(orc.BURGERS1D, nx, params=(0.05,))
    x = -1 + 2 * np.arange(nx) / nx
    u0 = 0.5 * np.sin(np.pi * x)
    rng = np.random.default_rng(5)
    M = 6 if corr == 0 else 40
    A, z = rng.uniform(-1, 1, (M, nx)), rng.uniform(-1, 1, M)

    def run(lam):
        return orc.parareal(pb, u0, N=N, t0=0.0, tN=0.4, F=(4, 40), G=(4, 2), eps=0.0, corr=corr,
                            net=orc.Net(A, z, orc.TANH, lam, 1.0), k_max=3, m_nn=3, keep_iterates=True)[1]

    i0 = run(0.0)
    assert i0["chol_fail"] == 0
    errs = [np.abs(run(lam)["U_iter"] - i0["U_iter"]).max() for lam in (1e-6, 1e-9)]
    assert errs[0] > errs[1] and errs[1] < 1e-6, errs
