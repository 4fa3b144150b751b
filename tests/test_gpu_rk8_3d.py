"""GPU: the eighth-order fine solver (Cooper and Verner's 11-stage method on
the generic propagator, every system) and the three-dimensional Brusselator
(App. E; seven-point periodic Laplacian, every propagator on the generic
form), through the C ABI against the CPU oracle."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2411_06225_amd as rpr  # noqa: E402
from paper_2411_06225_amd import workloads as W  # noqa: E402
from test_gpu_solve import E_err, assert_same_run  # noqa: E402


def initial_state(kind, nx, ny, nz, rng):
    nc = nx * ny * nz
    if kind == rpr.RPR_BURGERS1D:
        x = -1 + 2 * np.arange(nx) / nx
        return 0.5 * np.sin(np.pi * x) + 0.3 * np.cos(3 * np.pi * x) + 0.05 * rng.standard_normal(nx)
    if kind == rpr.RPR_DIFFREACT2D:
        return rng.standard_normal(2 * nc)
    if kind in (rpr.RPR_BRUSS2D, rpr.RPR_BRUSS3D):
        return np.concatenate([1 + 0.1 * rng.uniform(-1, 1, nc), 3 + 0.1 * rng.uniform(-1, 1, nc)])
    h = 1 + 0.1 * rng.random(nc)
    return np.concatenate([h, 0.05 * rng.standard_normal(nc), 0.05 * rng.standard_normal(nc)])


# (name, kind, nx, ny, nz, domain, params, steps, dt, method, threads)
GEN_CASES = [
    ("burgers_d128_rk8", rpr.RPR_BURGERS1D, 128, 1, 1, (-1, 1, -1, 1), (0.01,), 100, 1.5e-4, 8, 0),
    ("burgers_d100_rk8", rpr.RPR_BURGERS1D, 100, 1, 1, (-1, 1, -1, 1), (0.02,), 60, 1.5e-4, 8, 0),
    ("diffreact_13x9_rk8", rpr.RPR_DIFFREACT2D, 13, 9, 1, (-1, 1, -1, 1), (1e-3, 5e-3, 5e-3), 50, 1e-3, 8, 0),
    ("bruss_20x16_rk8", rpr.RPR_BRUSS2D, 20, 16, 1, (-1, 1, -1, 1), (1.0, 3.0, 0.02, 0.01), 50, 1e-3, 8, 0),
    ("swe_24x16_rk8", rpr.RPR_SWE2D, 24, 16, 1, (0, 1, 0, 1), (9.81,), 50, 5e-4, 8, 0),
    ("swe_24x16_rk4_generic", rpr.RPR_SWE2D, 24, 16, 1, (0, 1, 0, 1), (9.81,), 50, 5e-4, 4, 128),
    ("diffreact_40x30_rk1_generic", rpr.RPR_DIFFREACT2D, 40, 30, 1, (-1, 1, -1, 1), (1e-3, 5e-3, 5e-3), 20, 5e-3,
     1, 128),
    ("bruss3d_12x10x8_rk1", rpr.RPR_BRUSS3D, 12, 10, 8, (-1, 1, -1, 1), (1.0, 3.0, 0.1, 0.01), 20, 1e-3, 1, 0),
    ("bruss3d_12x10x8_rk4", rpr.RPR_BRUSS3D, 12, 10, 8, (-1, 1, -1, 1), (1.0, 3.0, 0.1, 0.01), 20, 2e-3, 4, 0),
    ("bruss3d_20_rk8", rpr.RPR_BRUSS3D, 20, 20, 20, (-1, 1, -1, 1), (1.0, 3.0, 0.1, 0.01), 10, 3e-3, 8, 0),
]


@pytest.mark.parametrize("case", GEN_CASES, ids=[c[0] for c in GEN_CASES])
@pytest.mark.parametrize("prec", [rpr.RPR_FP64, rpr.RPR_MIXED], ids=["fp64", "fp32"])
def test_generic_propagate_matches_oracle(orc, case, prec):
    """Three states per launch, odd and even step counts through the
    alternation of the stage inputs (and, with one stage, of the state)."""
    name, kind, nx, ny, nz, dom, params, steps, dt, method, threads = case
    rng = np.random.default_rng(abs(hash(name)) % 2 ** 32 + 3)
    X = np.stack([initial_state(kind, nx, ny, nz, rng) for _ in range(3)])
    d = X.shape[1]
    pb = orc.problem(kind, nx, ny, dom, params, nz=nz if kind == rpr.RPR_BRUSS3D else 0)
    h = rpr.make_rhs(kind, nx, ny, dom, params, nz=nz if kind == rpr.RPR_BRUSS3D else 0)
    dtype = torch.float64 if prec == rpr.RPR_FP64 else torch.float32
    for st in (steps, steps + 1):
        ref = orc.propagate_many(pb, method, st, dt, X)
        xin = torch.tensor(X, dtype=dtype, device="cuda")
        xout = torch.empty_like(xin)
        rpr.rpr_propagate(h, d, method, st, prec, dt, 3, xin, xout, threads=threads)
        torch.cuda.synchronize()
        got = xout.double().cpu().numpy()
        err = np.abs(got - ref).max() / np.abs(ref).max()
        print(name, "fp64" if prec == rpr.RPR_FP64 else "fp32", st, "rel err %.2e" % err)
        assert np.all(np.isfinite(got))
        assert err <= (1e-12 if prec == rpr.RPR_FP64 else 2e-5)


@pytest.mark.parametrize("method", [1, 4, 8])
def test_bruss3d_fixed_point_exact_on_gpu(method):
    nx, ny, nz = 9, 7, 5
    nc = nx * ny * nz
    h = rpr.make_rhs(rpr.RPR_BRUSS3D, nx, ny, params=(1.0, 3.0, 0.1, 0.01), nz=nz)
    x = torch.tensor(np.concatenate([np.full(nc, 1.0), np.full(nc, 3.0)])[None], device="cuda")
    y = torch.empty_like(x)
    rpr.rpr_propagate(h, 2 * nc, method, 9, rpr.RPR_FP64, 1e-3, 1, x, y)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(y.cpu().numpy(), x.cpu().numpy())


BRUSS3D_SMALL = W.BRUSS3D_20.replace(name="bruss3d_10", nx=10, ny=10, nz=10, N=8, tN=1.0, F=(8, 10), G=(1, 8), M=40)
BURGERS_RK8 = W.small(W.BURGERS_D128, nx=64, N=8, tN=2.0, F=(8, 100), G=(1, 20), M=32, params=(0.02,))


def gpu_solve3(w, corr=0, prec=0, k_max=0, **opt):
    A, z = W.random_weights(w)
    h = rpr.make_rhs(w.kind, w.nx, w.ny, w.domain, w.params, nz=w.nz if w.kind == rpr.RPR_BRUSS3D else 0)
    plan = rpr.Plan(h, w.d, w.t0, w.tN, w.N, F=w.F, G=w.G, tol=w.eps, M=w.M, activation=w.act, lam=w.lam, A=A,
                    zeta=z, precision=prec, correction=corr, k_max=k_max, **opt)
    U = torch.empty((w.N + 1, w.d), dtype=torch.float64, device="cuda")
    status = plan.execute(torch.tensor(W.initial_condition(w), dtype=torch.float64, device="cuda"), U)
    torch.cuda.synchronize()
    info = plan.info()
    info["status"] = status
    info["L_hist"], info["chg_hist"] = plan.history()
    plan.close()
    return U.cpu().numpy(), info


def orc_solve3(orc, w, corr=0, k_max=None, m_nn=4):
    pb = orc.problem(w.kind, w.nx, w.ny, w.domain, w.params, nz=w.nz if w.kind == rpr.RPR_BRUSS3D else 0)
    A, z = W.random_weights(w)
    return orc.parareal(pb, W.initial_condition(w), N=w.N, t0=w.t0, tN=w.tN, F=w.F, G=w.G, eps=w.eps, corr=corr,
                        net=orc.Net(A, z, w.act, w.lam, 0.0), k_max=k_max, m_nn=m_nn, nthreads=8)


SOLVES = [("bruss3d_10_global", BRUSS3D_SMALL, 0), ("bruss3d_10_nn", BRUSS3D_SMALL, 2),
          ("bruss3d_10_parareal", BRUSS3D_SMALL, 1), ("burgers_rk8_global", BURGERS_RK8, 0),
          ("burgers_rk8_nn", BURGERS_RK8, 2)]


@pytest.mark.parametrize("name,w,corr", SOLVES, ids=[s[0] for s in SOLVES])
def test_solve_matches_oracle(orc, name, w, corr):
    Ug, ig = gpu_solve3(w, corr=corr, stability=1)
    Uo, io = orc_solve3(orc, w, corr=corr)
    assert ig["unstable"] == 0
    if corr == 2:
        # the refit's forward error (as for the 2D nearest-neighbour solves)
        assert ig["K"] == io["K"] and ig["L_hist"].tolist() == io["L_hist"].tolist()
        assert np.abs(Ug - Uo).max() / np.abs(Uo).max() <= 1e-9
    else:
        assert_same_run(Ug, ig, Uo, io, w.N)


def test_bruss3d_reduced_precision_within_tau(orc):
    w = BRUSS3D_SMALL
    Ug, ig = gpu_solve3(w, prec=rpr.RPR_MIXED)
    pb = orc.problem(w.kind, w.nx, w.ny, w.domain, w.params, nz=w.nz)
    T = (w.tN - w.t0) / w.N
    Uf = orc.serial_fine(pb, w.F[0], w.F[1], T / w.F[1], w.N, W.initial_condition(w))
    Uo, _ = orc_solve3(orc, w, k_max=ig["K"])
    h = rpr.make_rhs(w.kind, w.nx, w.ny, w.domain, w.params, nz=w.nz)
    cur = torch.tensor(W.initial_condition(w), dtype=torch.float32, device="cuda")[None].contiguous()
    f32 = [cur[0].double().cpu().numpy()]
    for _ in range(w.N):
        nxt = torch.empty_like(cur)
        rpr.rpr_propagate(h, w.d, w.F[0], w.F[1], rpr.RPR_MIXED, T / w.F[1], 1, cur, nxt)
        cur = nxt
        f32.append(cur[0].double().cpu().numpy())
    tau = 10.0 * E_err(np.stack(f32), Uf)
    print("3D mixed K", ig["K"], "E %.2e FP64 E %.2e tau %.2e" % (E_err(Ug, Uf), E_err(Uo, Uf), tau))
    assert ig["converged"] == 1
    assert E_err(Ug, Uf) <= E_err(Uo, Uf) + tau


@pytest.mark.parametrize("form", ["graph", "segments"])
def test_bruss3d_sweep_forms_equal_the_cooperative_sweep(form):
    w = BRUSS3D_SMALL
    Ue, ie = gpu_solve3(w, sweep_form=1)
    opt = dict(graph=1, poll_every=2) if form == "graph" else dict(sweep_form=2)
    Ug, ig = gpu_solve3(w, **opt)
    assert ie["K"] == ig["K"]
    np.testing.assert_array_equal(Ug, Ue)
