"""RandNet-Parareal on AMD MI355X (gfx950).

Thin ctypes binding of ``librpr.so`` (C ABI in ``include/rpr.h``).  Every step
of the method runs in the library's HIP kernels; this module only marshals
arguments.  PyTorch is used for device memory and streams only.  If the built
library is missing, loading fails with an error: there is no CPU fallback.

Entry points keep the C names: ``rpr_plan_create``, ``rpr_plan_execute``,
``rpr_propagate``, ``rpr_randnet_features``, ``rpr_ridge_fit``,
``rpr_randnet_readout``, ``rpr_uniform_pm1`` ...; ``Plan`` and ``solve`` wrap
the plan calls for torch tensors.
"""
from __future__ import annotations

import atexit
import ctypes as C
import math
import os
import sys
import weakref

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librpr.so")

# status codes (rpr_status)
RPR_OK, RPR_NOT_CONVERGED = 0, 1
RPR_ERR_INVALID_ARG, RPR_ERR_NO_DEVICE, RPR_ERR_HIP, RPR_ERR_OOM = -1, -2, -3, -4
RPR_ERR_NONFINITE, RPR_ERR_NOT_SPD, RPR_ERR_UNSTABLE, RPR_ERR_UNSUPPORTED = -5, -6, -7, -8
# enums
RPR_BURGERS1D, RPR_DIFFREACT2D, RPR_BRUSS2D, RPR_SWE2D, RPR_BRUSS3D = 0, 1, 2, 3, 4
RPR_RK1, RPR_RK4, RPR_RK8 = 1, 4, 8
RPR_TANH, RPR_RELU = 0, 1
RPR_FP64, RPR_MIXED = 0, 1
RPR_CORR_RANDNET, RPR_CORR_PARAREAL, RPR_CORR_RANDNET_NN = 0, 1, 2
RPR_FEAT_AUTO, RPR_FEAT_FP64, RPR_FEAT_BF16 = 0, 1, 2

EXPORTED = ("rpr_last_error", "rpr_version", "rpr_plan_create", "rpr_plan_execute", "rpr_plan_info",
            "rpr_plan_history", "rpr_plan_destroy", "rpr_propagate", "rpr_randnet_features", "rpr_ridge_fit",
            "rpr_randnet_readout", "rpr_uniform_pm1", "rpr_randnet_features_bf16", "rpr_plan_create_batch",
            "rpr_plan_execute_batch", "rpr_plan_instance", "rpr_stability", "rpr_randnet_features_noalloc",
            "rpr_tune_set", "rpr_tune_get", "rpr_tile_shapes", "rpr_tile_shape_name")


class RprError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"rpr status {status}: {msg}")
        self.status = status


class rpr_rhs(C.Structure):
    _fields_ = [("kind", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("x0", C.c_double), ("x1", C.c_double), ("y0", C.c_double), ("y1", C.c_double),
                ("p", C.c_double * 6)]


class rpr_propagator(C.Structure):
    _fields_ = [("method", C.c_int32), ("threads", C.c_int32), ("steps", C.c_int64)]


class rpr_randnet(C.Structure):
    _fields_ = [("M", C.c_int32), ("activation", C.c_int32), ("lam", C.c_double), ("input_scale", C.c_double),
                ("m_nn", C.c_int32), ("reserved", C.c_int32)]


class rpr_options(C.Structure):
    _fields_ = [("precision", C.c_int32), ("correction", C.c_int32), ("k_max", C.c_int32),
                ("poll_every", C.c_int32), ("features", C.c_int32), ("autotune", C.c_int32),
                ("graph", C.c_int32), ("stability", C.c_int32), ("chain_wgs", C.c_int32), ("sweep_form", C.c_int32)]


class rpr_info(C.Structure):
    _fields_ = [("K", C.c_int32), ("L_final", C.c_int32), ("converged", C.c_int32), ("rows_used", C.c_int32),
                ("nonfinite_rows", C.c_int32), ("chol_fail", C.c_int32), ("input_scale", C.c_double),
                ("t_total", C.c_double), ("t_fine", C.c_double), ("t_model", C.c_double), ("t_sweep", C.c_double),
                ("stab_F", C.c_double), ("stab_G", C.c_double), ("unstable", C.c_int32), ("reserved", C.c_int32)]


_lib = None
# Plans still open: closed before the interpreter shuts down, so that no plan
# is released from a finaliser after the HIP runtime has begun its own
# teardown.
_live = weakref.WeakSet()


_exiting = [False]


@atexit.register
def _close_live_plans():
    _exiting[0] = True
    for plan in list(_live):
        try:
            plan.close()
        except Exception:
            pass


def lib() -> C.CDLL:
    """The loaded librpr.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        # PyTorch ships its own HIP runtime under the same soname as the
        # system's; importing it first makes the process load that one, and
        # librpr binds to it (loaded the other way round, torch and librpr
        # end up with runtimes that do not share the device)
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2411_06225_amd.build` "
                              "(there is no CPU fallback)")
        L = C.CDLL(LIB_PATH)
        vp, dp, i32, i64, u64, dbl = C.c_void_p, C.POINTER(C.c_double), C.c_int32, C.c_int64, C.c_uint64, C.c_double
        sig = {
            "rpr_last_error": (C.c_char_p, []),
            "rpr_version": (C.c_char_p, []),
            "rpr_plan_create": (i32, [C.POINTER(vp), C.POINTER(rpr_rhs), i32, dbl, dbl, i32,
                                      C.POINTER(rpr_propagator), C.POINTER(rpr_propagator), dbl,
                                      C.POINTER(rpr_randnet), vp, vp, u64, C.POINTER(rpr_options)]),
            "rpr_plan_execute": (i32, [vp, vp, vp, vp]),
            "rpr_plan_create_batch": (i32, [C.POINTER(vp), i32, C.POINTER(rpr_rhs), C.POINTER(C.c_int32), dp, dp,
                                            C.POINTER(C.c_int32), C.POINTER(rpr_propagator),
                                            C.POINTER(rpr_propagator), dp, C.POINTER(rpr_randnet),
                                            C.POINTER(vp), C.POINTER(vp), u64, C.POINTER(rpr_options)]),
            "rpr_plan_execute_batch": (i32, [vp, C.POINTER(vp), C.POINTER(vp), vp]),
            "rpr_plan_instance": (i32, [vp, i32, C.POINTER(vp)]),
            "rpr_plan_info": (i32, [vp, C.POINTER(rpr_info)]),
            "rpr_plan_history": (i32, [vp, C.POINTER(C.c_int32), dp, i32]),
            "rpr_plan_destroy": (i32, [vp]),
            "rpr_propagate": (i32, [C.POINTER(rpr_rhs), i32, C.POINTER(rpr_propagator), i32, dbl, i32, vp, vp,
                                    vp]),
            "rpr_randnet_features": (i32, [i32, i32, i32, i32, dbl, vp, vp, vp, vp, vp]),
            "rpr_randnet_features_bf16": (i32, [i32, i32, i32, i32, dbl, vp, vp, vp, vp, vp]),
            "rpr_randnet_features_noalloc": (i32, [i32, i32, i32, i32, dbl, vp, vp, vp, vp, vp]),
            "rpr_ridge_fit": (i32, [i32, i32, i32, vp, vp, dbl, vp, vp]),
            "rpr_randnet_readout": (i32, [i32, i32, i32, vp, vp, vp, vp]),
            "rpr_uniform_pm1": (i32, [u64, u64, i64, vp, vp]),
            "rpr_stability": (i32, [C.POINTER(rpr_rhs), i32, C.POINTER(rpr_propagator), dbl, dbl, dbl, dp]),
            "rpr_tune_set": (i32, [C.c_char_p, i32]),
            "rpr_tune_get": (i32, [C.c_char_p, C.POINTER(C.c_int32)]),
            "rpr_tile_shapes": (i32, [i32, i32]),
            "rpr_tile_shape_name": (C.c_char_p, [i32, i32, i32]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def last_error() -> str:
    return lib().rpr_last_error().decode()


def check(status: int, allow=(RPR_OK,)) -> int:
    if status not in allow:
        raise RprError(status, last_error())
    return status


def _ptr(t) -> int | None:
    """Address of a torch tensor, an int (a raw pointer, passed through
    unchecked), or None."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _dev(t, dtype: str, numel: int, name: str) -> int | None:
    """Address of a device tensor after checking what the C ABI assumes of it:
    a CUDA tensor of the given dtype ("float64" or "float32"), contiguous, with
    at least `numel` elements.  Raw integer pointers pass through unchecked."""
    if t is None or isinstance(t, int):
        return _ptr(t)
    import torch
    want = getattr(torch, dtype)
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name}: expected a torch tensor or an int pointer, got {type(t).__name__}")
    if not t.is_cuda:
        raise ValueError(f"{name}: must be a device (cuda) tensor")
    if t.dtype != want:
        raise TypeError(f"{name}: dtype {t.dtype}, expected {want}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")
    if t.numel() < numel:
        raise ValueError(f"{name}: {t.numel()} elements, at least {numel} needed")
    return t.data_ptr()


def _stream(stream) -> int | None:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return stream if isinstance(stream, int) else stream.cuda_stream


def make_rhs(kind: int, nx: int, ny: int = 1, domain=(-1.0, 1.0, -1.0, 1.0), params=(), nz: int = 0) -> rpr_rhs:
    p = (C.c_double * 6)(*([float(v) for v in params] + [0.0] * (6 - len(params))))
    x0, x1, y0, y1 = (float(v) for v in domain)
    return rpr_rhs(int(kind), int(nx), int(ny), int(nz), x0, x1, y0, y1, p)


def nspecies(kind: int) -> int:
    return {RPR_BURGERS1D: 1, RPR_DIFFREACT2D: 2, RPR_BRUSS2D: 2, RPR_SWE2D: 3, RPR_BRUSS3D: 2}[kind]


# ---- building blocks ---------------------------------------------------------
def rpr_propagate(h: rpr_rhs, d: int, method: int, steps: int, precision: int, dt: float, n_states: int, x_in,
                  x_out, stream=None, threads: int = 0) -> int:
    P = rpr_propagator(int(method), int(threads), int(steps))
    dt_ = "float64" if precision == RPR_FP64 else "float32"
    n = int(n_states) * int(d)
    return check(lib().rpr_propagate(C.byref(h), int(d), C.byref(P), int(precision), float(dt), int(n_states),
                                     _dev(x_in, dt_, n, "x_in"), _dev(x_out, dt_, n, "x_out"), _stream(stream)))


def rpr_randnet_features(M: int, d: int, n: int, activation: int, s: float, A, zeta, X, Phi, stream=None) -> int:
    return check(lib().rpr_randnet_features(int(M), int(d), int(n), int(activation), float(s),
                                            _dev(A, "float64", M * d, "A"), _dev(zeta, "float64", M, "zeta"),
                                            _dev(X, "float64", n * d, "X"), _dev(Phi, "float64", n * M, "Phi"),
                                            _stream(stream)))


def rpr_randnet_features_noalloc(M: int, d: int, n: int, activation: int, s: float, A, zeta, X, Phi,
                                 stream=None) -> int:
    return check(lib().rpr_randnet_features_noalloc(int(M), int(d), int(n), int(activation), float(s),
                                                    _dev(A, "float64", M * d, "A"), _dev(zeta, "float64", M, "zeta"),
                                                    _dev(X, "float64", n * d, "X"), _dev(Phi, "float64", n * M, "Phi"),
                                                    _stream(stream)))


def rpr_randnet_features_bf16(M: int, d: int, n: int, activation: int, s: float, A, zeta, X, Phi,
                              stream=None) -> int:
    return check(lib().rpr_randnet_features_bf16(int(M), int(d), int(n), int(activation), float(s),
                                                 _dev(A, "float64", M * d, "A"), _dev(zeta, "float64", M, "zeta"),
                                                 _dev(X, "float32", n * d, "X"), _dev(Phi, "float64", n * M, "Phi"),
                                                 _stream(stream)))


def rpr_ridge_fit(M: int, d: int, n: int, Phi, Y, lam: float, W, stream=None) -> int:
    return check(lib().rpr_ridge_fit(int(M), int(d), int(n), _dev(Phi, "float64", n * M, "Phi"),
                                     _dev(Y, "float64", n * d, "Y"), float(lam), _dev(W, "float64", M * d, "W"),
                                     _stream(stream)))


def rpr_randnet_readout(M: int, d: int, n: int, W, Phi, Yhat, stream=None) -> int:
    return check(lib().rpr_randnet_readout(int(M), int(d), int(n), _dev(W, "float64", M * d, "W"),
                                           _dev(Phi, "float64", n * M, "Phi"), _dev(Yhat, "float64", n * d, "Yhat"),
                                           _stream(stream)))


def rpr_uniform_pm1(seed: int, first: int, n: int, out, stream=None) -> int:
    return check(lib().rpr_uniform_pm1(C.c_uint64(seed), C.c_uint64(first), int(n), _dev(out, "float64", n, "out"),
                                       _stream(stream)))


def rpr_stability(h: rpr_rhs, d: int, method: int, steps: int, dt: float, umax: float, speed: float = 0.0) -> float:
    """dt / dt_max of one propagator at a state with max |u| = umax (host only)."""
    P = rpr_propagator(int(method), 0, int(steps))
    r = C.c_double(0.0)
    check(lib().rpr_stability(C.byref(h), int(d), C.byref(P), float(dt), float(umax), float(speed), C.byref(r)))
    return r.value


def rpr_tune_set(key: str, value: int) -> int:
    """Store a launch shape in the autotuner's table (value < 0 removes the key)."""
    return check(lib().rpr_tune_set(key.encode(), int(value)))


def rpr_tune_get(key: str):
    """The launch shape stored under key, or None."""
    v = C.c_int32(0)
    return v.value if lib().rpr_tune_get(key.encode(), C.byref(v)) == 0 else None


def tile_shapes(kind: int, precision: int) -> list:
    """Names of the one-pass RK4 kernel's tile shapes, in index order."""
    L = lib()
    return [L.rpr_tile_shape_name(int(kind), int(precision), v).decode()
            for v in range(L.rpr_tile_shapes(int(kind), int(precision)))]


def prop_tune_key(kind: int, nx: int, ny: int, precision: int, method: int) -> str:
    """Table key of the fine propagator's class (append ":v" for the tile shape)."""
    return f"prop:{int(kind)}:{int(nx)}x{int(ny)}:{8 if precision == RPR_FP64 else 4}:{int(method)}"


def chain_tune_key(kind: int, nx: int, ny: int, precision: int, M: int, N: int, correction: int = 0,
                   bf16_features: bool | None = None) -> str:
    """Table key of a plan's sweep (append ":B" for its work-group size)."""
    f = (precision == RPR_MIXED) if bf16_features is None else bf16_features
    return (f"chain:{int(kind)}:{int(nx)}x{int(ny)}:{8 if precision == RPR_FP64 else 4}:M{int(M)}:N{int(N)}:"
            f"{int(correction)}:{1 if f else 0}")


# ---- plans ---------------------------------------------------------------------
class Plan:
    """One IVP solved by RandNet-Parareal (rpr_plan_create / execute / destroy)."""

    def __init__(self, h: rpr_rhs, d: int, t0: float, tN: float, N: int, F=(RPR_RK4, 1), G=(RPR_RK1, 1),
                 tol: float = 1e-6, M: int = 100, activation: int = RPR_TANH, lam: float = 1e-6,
                 input_scale: float = 0.0, A=None, zeta=None, seed: int = 0, precision: int = RPR_FP64,
                 correction: int = RPR_CORR_RANDNET, k_max: int = 0, poll_every: int = 0,
                 features: int = RPR_FEAT_AUTO, autotune: int = 0, graph: int = 0, m_nn: int = 4,
                 stability: int = 0, chain_wgs: int = 0, sweep_form: int = 0):
        import numpy as np
        self.d, self.N = int(d), int(N)
        # F, G: (method, steps) or (method, steps, threads)
        self._F = rpr_propagator(int(F[0]), int(F[2]) if len(F) > 2 else 0, int(F[1]))
        self._G = rpr_propagator(int(G[0]), int(G[2]) if len(G) > 2 else 0, int(G[1]))
        self._net = rpr_randnet(int(M), int(activation), float(lam), float(input_scale), int(m_nn), 0)
        self._opt = rpr_options(int(precision), int(correction), int(k_max), int(poll_every), int(features),
                                int(autotune), int(graph), int(stability), int(chain_wgs), int(sweep_form))
        self._h = h
        Ah = zh = None
        if A is not None:
            Ah = np.ascontiguousarray(A, dtype=np.float64)
            zh = np.ascontiguousarray(zeta, dtype=np.float64)
        self._handle = C.c_void_p()
        _live.add(self)
        check(lib().rpr_plan_create(C.byref(self._handle), C.byref(h), self.d, float(t0), float(tN), self.N,
                                    C.byref(self._F), C.byref(self._G), float(tol), C.byref(self._net),
                                    None if Ah is None else Ah.ctypes.data, None if zh is None else zh.ctypes.data,
                                    C.c_uint64(seed), C.byref(self._opt)))

    def execute(self, u0, U_out, stream=None) -> int:
        """u0: cuda float64 tensor (d); U_out: cuda float64 tensor ((N+1) x d)."""
        return check(lib().rpr_plan_execute(self._handle, _dev(u0, "float64", self.d, "u0"),
                                            _dev(U_out, "float64", (self.N + 1) * self.d, "U_out"), _stream(stream)),
                     allow=(RPR_OK, RPR_NOT_CONVERGED))

    def info(self) -> dict:
        inf = rpr_info()
        check(lib().rpr_plan_info(self._handle, C.byref(inf)))
        return {k: getattr(inf, k) for k, _ in rpr_info._fields_}

    def history(self):
        import numpy as np
        L = np.zeros(self.N + 1, dtype=np.int32)
        ch = np.zeros(self.N + 1)
        check(lib().rpr_plan_history(self._handle, L.ctypes.data_as(C.POINTER(C.c_int32)),
                                     ch.ctypes.data_as(C.POINTER(C.c_double)), self.N + 1))
        K = self.info()["K"]
        return L[:K + 1], ch[:K + 1]

    def close(self):
        if self._handle:
            lib().rpr_plan_destroy(self._handle)
            self._handle = C.c_void_p()

    def __del__(self):
        try:
            if _exiting[0]:
                return  # the exit hook has closed every plan already
            self.close()
        except Exception:  # module globals already torn down
            pass


class _Handle:
    """Instance view of a batch (info / history only)."""

    def __init__(self, handle, N):
        self._handle, self.N = handle, N

    info = Plan.info
    history = Plan.history


class BatchPlan:
    """Many independent IVPs solved together (rpr_plan_create_batch / execute_batch)."""

    def __init__(self, problems, *, tol=1e-6, precision: int = RPR_FP64, correction: int = RPR_CORR_RANDNET,
                 k_max: int = 0, poll_every: int = 0, features: int = RPR_FEAT_AUTO, seed: int = 0, graph: int = 0,
                 stability: int = 0, autotune: int = 0):
        """problems: list of dicts with keys h, d, t0, tN, N, F, G, M, activation, lam, A, zeta
        (and m_nn for RPR_CORR_RANDNET_NN, default 4)."""
        import numpy as np
        n = len(problems)
        self.n = n
        self.Ns = [int(q["N"]) for q in problems]
        self.ds = [int(q["d"]) for q in problems]
        H = (rpr_rhs * n)(*[q["h"] for q in problems])
        D = (C.c_int32 * n)(*self.ds)
        T0 = (C.c_double * n)(*[float(q["t0"]) for q in problems])
        TN = (C.c_double * n)(*[float(q["tN"]) for q in problems])
        NN = (C.c_int32 * n)(*self.Ns)
        F = (rpr_propagator * n)(*[rpr_propagator(int(q["F"][0]), 0, int(q["F"][1])) for q in problems])
        G = (rpr_propagator * n)(*[rpr_propagator(int(q["G"][0]), 0, int(q["G"][1])) for q in problems])
        TOL = (C.c_double * n)(*([float(tol)] * n if not isinstance(tol, (list, tuple)) else [float(t) for t in tol]))
        NET = (rpr_randnet * n)(*[rpr_randnet(int(q.get("M", 100)), int(q.get("activation", RPR_TANH)),
                                              float(q.get("lam", 1e-6)), float(q.get("input_scale", 0.0)),
                                              int(q.get("m_nn", 4)), 0)
                                  for q in problems])
        self._keep = []
        Ap = (C.c_void_p * n)()
        Zp = (C.c_void_p * n)()
        have = all(q.get("A") is not None for q in problems)
        if have:
            for b, q in enumerate(problems):
                a = np.ascontiguousarray(q["A"], dtype=np.float64)
                z = np.ascontiguousarray(q["zeta"], dtype=np.float64)
                self._keep += [a, z]
                Ap[b], Zp[b] = a.ctypes.data, z.ctypes.data
        opt = rpr_options(int(precision), int(correction), int(k_max), int(poll_every), int(features), int(autotune),
                          int(graph), int(stability), 0, 0)
        self._handle = C.c_void_p()
        _live.add(self)
        check(lib().rpr_plan_create_batch(C.byref(self._handle), n, H, D, T0, TN, NN, F, G, TOL, NET,
                                          Ap if have else None, Zp if have else None, C.c_uint64(seed),
                                          C.byref(opt)))

    def execute(self, u0s, U_outs, stream=None) -> int:
        n = self.n
        if len(u0s) != n or len(U_outs) != n:
            raise ValueError(f"need {n} initial states and {n} outputs")
        U0 = (C.c_void_p * n)(*[_dev(u, "float64", self.ds[b], f"u0[{b}]") for b, u in enumerate(u0s)])
        UO = (C.c_void_p * n)(*[_dev(u, "float64", (self.Ns[b] + 1) * self.ds[b], f"U_out[{b}]")
                                for b, u in enumerate(U_outs)])
        return check(lib().rpr_plan_execute_batch(self._handle, U0, UO, _stream(stream)),
                     allow=(RPR_OK, RPR_NOT_CONVERGED))

    def instance(self, b: int) -> "_Handle":
        h = C.c_void_p()
        check(lib().rpr_plan_instance(self._handle, int(b), C.byref(h)))
        return _Handle(h, self.Ns[b])

    def close(self):
        if self._handle:
            lib().rpr_plan_destroy(self._handle)
            self._handle = C.c_void_p()

    def __del__(self):
        try:
            if _exiting[0]:
                return  # the exit hook has closed every plan already
            self.close()
        except Exception:  # module globals already torn down
            pass


def solve(h: rpr_rhs, u0, *, t0: float, tN: float, N: int, **kw):
    """Solve with a fresh plan; returns (U (N+1) x d cuda float64 tensor, info dict)."""
    import torch
    d = u0.numel()
    plan = Plan(h, d, t0, tN, N, **kw)
    U = torch.empty((N + 1, d), dtype=torch.float64, device=u0.device)
    plan.execute(u0, U)
    torch.cuda.synchronize()
    info = plan.info()
    info["L_hist"], info["chg_hist"] = plan.history()
    plan.close()
    return U, info
