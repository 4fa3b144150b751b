"""Plain serial FP64 CPU oracle for RandNet-Parareal (arXiv 2411.06225).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this package.  It wraps ``liboracle.so``
(built from the C sources beside this file with gcc, no FMA contraction) and
shares no code with the GPU library.

Every function cites the part of the paper it follows in the C source; this
module only marshals numpy arrays.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SOURCES = ["rhs.c", "integrate.c", "randnet.c", "parareal.c", "stability.c"]

BURGERS1D, DIFFREACT2D, BRUSS2D, SWE2D, BRUSS3D = 0, 1, 2, 3, 4
TANH, RELU = 0, 1
CORR_RANDNET, CORR_PARAREAL, CORR_RANDNET_NN = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (plain -O2, no contraction, no fast-math)."""
    if not force and os.path.exists(_LIB_PATH):
        return _LIB_PATH
    cmd = ["gcc", "-O2", "-std=c99", "-D_POSIX_C_SOURCE=200809L", "-fPIC", "-shared",
           "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wno-unused-function",
           "-o", _LIB_PATH + ".tmp"] + [os.path.join(_HERE, s) for s in _SOURCES] + ["-lm", "-lpthread"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


class Problem(C.Structure):
    _fields_ = [("kind", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("x0", C.c_double), ("x1", C.c_double), ("y0", C.c_double), ("y1", C.c_double),
                ("p", C.c_double * 6)]


class RandNet(C.Structure):
    _fields_ = [("M", C.c_int32), ("act", C.c_int32), ("lam", C.c_double), ("scale", C.c_double),
                ("A", C.POINTER(C.c_double)), ("zeta", C.POINTER(C.c_double))]


class Info(C.Structure):
    _fields_ = [("K", C.c_int32), ("L_final", C.c_int32), ("converged", C.c_int32),
                ("rows_used", C.c_int32), ("nonfinite_rows", C.c_int32), ("chol_fail", C.c_int32)]


class PararealCfg(C.Structure):
    _fields_ = [("N", C.c_int32), ("F_method", C.c_int32), ("G_method", C.c_int32),
                ("corr", C.c_int32), ("F_steps", C.c_int64), ("G_steps", C.c_int64),
                ("t0", C.c_double), ("tN", C.c_double), ("eps", C.c_double),
                ("k_max", C.c_int32), ("m_nn", C.c_int32), ("nthreads", C.c_int32),
                ("pad", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = C.CDLL(_LIB_PATH)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int32)
        L.orc_dim.restype = C.c_int32
        L.orc_dim.argtypes = [C.POINTER(Problem)]
        L.orc_rhs.restype = C.c_int32
        L.orc_rhs.argtypes = [C.POINTER(Problem), dp, dp]
        L.orc_propagate.restype = C.c_int32
        L.orc_propagate.argtypes = [C.POINTER(Problem), C.c_int32, C.c_int64, C.c_double, dp, dp]
        L.orc_propagate_many.restype = C.c_int32
        L.orc_propagate_many.argtypes = [C.POINTER(Problem), C.c_int32, C.c_int64, C.c_double,
                                         C.c_int32, dp, dp, C.c_int32]
        L.orc_serial_fine.restype = C.c_int32
        L.orc_serial_fine.argtypes = [C.POINTER(Problem), C.c_int32, C.c_int64, C.c_double,
                                      C.c_int32, dp, dp]
        L.orc_features.restype = None
        L.orc_features.argtypes = [C.POINTER(RandNet), C.c_int32, C.c_int32, dp, dp]
        L.orc_ridge_fit.restype = C.c_int32
        L.orc_ridge_fit.argtypes = [C.c_int32, C.c_int32, C.c_int32, dp, dp, C.c_double, dp]
        L.orc_ridge_fit_dual.restype = C.c_int32
        L.orc_ridge_fit_dual.argtypes = [C.c_int32, C.c_int32, C.c_int32, dp, dp, C.c_double, dp]
        L.orc_cholesky.restype = C.c_int32
        L.orc_cholesky.argtypes = [C.c_int32, dp, dp]
        L.orc_ridgeless_fit.restype = C.c_int32
        L.orc_ridgeless_fit.argtypes = [C.c_int32, C.c_int32, C.c_int32, dp, dp, dp, C.POINTER(C.c_int32)]
        L.orc_ridgeless_stats.restype = C.c_int32
        L.orc_ridgeless_stats.argtypes = [C.c_int32, C.c_int32, C.c_int32, dp, dp, dp, C.POINTER(C.c_int32)]
        L.orc_sym_eig.restype = None
        L.orc_sym_eig.argtypes = [C.c_int32, dp, dp, dp]
        L.orc_nearest.restype = None
        L.orc_nearest.argtypes = [C.c_int32, C.c_int32, dp, dp, C.c_int32, ip]
        L.orc_splitmix64.restype = C.c_uint64
        L.orc_splitmix64.argtypes = [C.c_uint64, C.c_uint64]
        L.orc_uniform_pm1.restype = None
        L.orc_uniform_pm1.argtypes = [C.c_uint64, C.c_uint64, C.c_int64, dp]
        L.orc_rk_tableau.restype = C.c_int32
        L.orc_rk_tableau.argtypes = [C.c_int32, C.POINTER(C.c_int32), dp, dp, dp]
        L.orc_stability.restype = C.c_double
        L.orc_stability.argtypes = [C.POINTER(Problem), C.c_int32, C.c_double, dp]
        L.orc_input_scale.restype = C.c_double
        L.orc_input_scale.argtypes = [C.c_int32, dp]
        L.orc_parareal.restype = C.c_int32
        L.orc_parareal.argtypes = [C.POINTER(Problem), C.POINTER(PararealCfg), C.POINTER(RandNet),
                                   dp, dp, ip, dp, dp, C.POINTER(Info)]
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def problem(kind: int, nx: int, ny: int = 1, domain=(-1.0, 1.0, -1.0, 1.0), params=(), nz: int = 0) -> Problem:
    p = (C.c_double * 6)(*([float(v) for v in params] + [0.0] * (6 - len(params))))
    x0, x1, y0, y1 = (float(v) for v in domain)
    return Problem(int(kind), int(nx), int(ny), int(nz), x0, x1, y0, y1, p)


def rk_tableau(method: int):
    """(A, b, c) of the oracle's explicit Runge-Kutta method `method`."""
    s = C.c_int32(0)
    A, b, c = np.zeros(256), np.zeros(16), np.zeros(16)
    if lib().orc_rk_tableau(int(method), C.byref(s), _dp(A), _dp(b), _dp(c)):
        raise ValueError(f"no tableau for method {method}")
    n = s.value
    return A[: n * n].reshape(n, n).copy(), b[:n].copy(), c[:n].copy()


def dim(pb: Problem) -> int:
    return int(lib().orc_dim(C.byref(pb)))


def rhs(pb: Problem, u) -> np.ndarray:
    u = _f64(u)
    out = np.empty_like(u)
    rc = lib().orc_rhs(C.byref(pb), _dp(u), _dp(out))
    if rc:
        raise ValueError(f"orc_rhs failed ({rc})")
    return out


def propagate(pb: Problem, method: int, steps: int, dt: float, u) -> np.ndarray:
    u = _f64(u)
    out = np.empty_like(u)
    rc = lib().orc_propagate(C.byref(pb), int(method), int(steps), float(dt), _dp(u), _dp(out))
    if rc:
        raise ValueError(f"orc_propagate failed ({rc})")
    return out


def propagate_many(pb: Problem, method: int, steps: int, dt: float, X, nthreads: int = 1) -> np.ndarray:
    X = _f64(X)
    out = np.empty_like(X)
    rc = lib().orc_propagate_many(C.byref(pb), int(method), int(steps), float(dt), X.shape[0],
                                  _dp(X), _dp(out), int(nthreads))
    if rc:
        raise ValueError(f"orc_propagate_many failed ({rc})")
    return out


def serial_fine(pb: Problem, method: int, steps: int, dt: float, N: int, u0) -> np.ndarray:
    u0 = _f64(u0)
    U = np.empty((N + 1, u0.size))
    rc = lib().orc_serial_fine(C.byref(pb), int(method), int(steps), float(dt), int(N), _dp(u0), _dp(U))
    if rc:
        raise ValueError(f"orc_serial_fine failed ({rc})")
    return U


class Net:
    """Keeps the numpy arrays of a RandNet alive next to its ctypes struct."""

    def __init__(self, A, zeta, act: int, lam: float, scale: float):
        self.A = _f64(A)
        self.zeta = _f64(zeta)
        self.st = RandNet(self.A.shape[0], int(act), float(lam), float(scale), _dp(self.A), _dp(self.zeta))


def features(net: Net, X) -> np.ndarray:
    X = np.atleast_2d(_f64(X))
    out = np.empty((X.shape[0], net.A.shape[0]))
    lib().orc_features(C.byref(net.st), X.shape[1], X.shape[0], _dp(X), _dp(out))
    return out


def ridge_fit(Phi, Y, lam: float) -> np.ndarray:
    Phi, Y = _f64(Phi), _f64(Y)
    W = np.empty((Phi.shape[1], Y.shape[1]))
    rc = lib().orc_ridge_fit(Phi.shape[1], Y.shape[1], Phi.shape[0], _dp(Phi), _dp(Y), float(lam), _dp(W))
    if rc:
        raise np.linalg.LinAlgError(f"orc_ridge_fit failed ({rc})")
    return W


def ridgeless_fit(Phi, Y):
    """eq. "ridgeless" at lambda -> 0: W = Phi^+ Y, and the rank of the Gram."""
    Phi, Y = _f64(Phi), _f64(Y)
    W = np.empty((Phi.shape[1], Y.shape[1]))
    r = C.c_int32(0)
    lib().orc_ridgeless_fit(Phi.shape[1], Y.shape[1], Phi.shape[0], _dp(Phi), _dp(Y), _dp(W), C.byref(r))
    return W, r.value


def ridgeless_stats(G, B, n: int):
    """The same limit from G = Phi^T Phi and B = Phi^T Y of n rows: W = G^+ B, rank."""
    G, B = _f64(G), _f64(B)
    W = np.empty_like(B)
    r = C.c_int32(0)
    lib().orc_ridgeless_stats(G.shape[0], B.shape[1], int(n), _dp(G), _dp(B), _dp(W), C.byref(r))
    return W, r.value


def sym_eig(S):
    """Eigenvalues and eigenvectors (columns) of a symmetric matrix, cyclic Jacobi."""
    S = _f64(S)
    w, V = np.empty(S.shape[0]), np.empty_like(S)
    lib().orc_sym_eig(S.shape[0], _dp(S), _dp(w), _dp(V))
    return w, V


def ridge_fit_dual(Phi, Y, lam: float) -> np.ndarray:
    Phi, Y = _f64(Phi), _f64(Y)
    W = np.empty((Phi.shape[1], Y.shape[1]))
    rc = lib().orc_ridge_fit_dual(Phi.shape[1], Y.shape[1], Phi.shape[0], _dp(Phi), _dp(Y), float(lam), _dp(W))
    if rc:
        raise np.linalg.LinAlgError(f"orc_ridge_fit_dual failed ({rc})")
    return W


def cholesky(S) -> np.ndarray:
    S = _f64(S)
    L = np.empty_like(S)
    rc = lib().orc_cholesky(S.shape[0], _dp(S), _dp(L))
    if rc:
        raise np.linalg.LinAlgError("orc_cholesky: not positive definite")
    return L


def nearest(P, q, m: int) -> np.ndarray:
    P, q = _f64(P), _f64(q)
    idx = np.empty(m, dtype=np.int32)
    lib().orc_nearest(P.shape[1], P.shape[0], _dp(P), _dp(q), int(m),
                      idx.ctypes.data_as(C.POINTER(C.c_int32)))
    return idx


def splitmix64(seed: int, i: int) -> int:
    return int(lib().orc_splitmix64(C.c_uint64(seed), C.c_uint64(i)))


def uniform_pm1(seed: int, first: int, n: int) -> np.ndarray:
    out = np.empty(n)
    lib().orc_uniform_pm1(C.c_uint64(seed), C.c_uint64(first), int(n), _dp(out))
    return out


def stability(pb: Problem, method: int, dt: float, u) -> float:
    """dt / dt_max of the propagator `method` for h linearised at u."""
    u = _f64(u)
    return float(lib().orc_stability(C.byref(pb), int(method), float(dt), _dp(u)))


def input_scale(u0) -> float:
    """The default input scale of the random network for initial state u0."""
    u0 = _f64(u0)
    return float(lib().orc_input_scale(u0.size, _dp(u0)))


def parareal(pb: Problem, u0, *, N: int, t0: float, tN: float, F=(4, 1), G=(1, 1), eps: float,
             corr: int = CORR_RANDNET, net: Net | None = None, k_max: int | None = None,
             m_nn: int = 4, nthreads: int = 1, keep_iterates: bool = False):
    """Runs the oracle's Parareal iteration.

    F and G are (method, steps per slice).  Returns (U, info) where U is
    (N+1) x d and info a dict with K, L history, change history and counters;
    with keep_iterates the dict also holds ``U_iter`` ((k_max+1) x (N+1) x d).
    """
    u0 = _f64(u0)
    d = u0.size
    k_max = N if k_max is None else int(k_max)
    cfg = PararealCfg(int(N), int(F[0]), int(G[0]), int(corr), int(F[1]), int(G[1]), float(t0),
                      float(tN), float(eps), k_max, int(m_nn), int(nthreads), 0)
    U = np.empty((N + 1, d))
    L_hist = np.zeros(k_max + 1, dtype=np.int32)
    chg = np.zeros(k_max + 1)
    U_iter = np.zeros((k_max + 1, N + 1, d)) if keep_iterates else None
    info = Info()
    rc = lib().orc_parareal(C.byref(pb), C.byref(cfg), C.byref(net.st) if net is not None else None,
                            _dp(u0), _dp(U), L_hist.ctypes.data_as(C.POINTER(C.c_int32)), _dp(chg),
                            _dp(U_iter) if keep_iterates else None, C.byref(info))
    if rc:
        raise RuntimeError(f"orc_parareal failed ({rc})")
    K = info.K
    out = dict(K=K, L_final=info.L_final, converged=bool(info.converged), rows_used=info.rows_used,
               nonfinite_rows=info.nonfinite_rows, chol_fail=info.chol_fail,
               L_hist=L_hist[:K + 1].copy(), chg_hist=chg[:K + 1].copy())
    if keep_iterates:
        out["U_iter"] = U_iter[:K + 1]
    return U, out
