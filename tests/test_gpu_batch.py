"""GPU batches: many independent IVPs of uneven size in one plan, against the
oracle solving each instance on its own.  The persistent fine-solve launch and
the one-work-group-per-instance chain must not change any instance's run:
same iteration count and L history, states within N * 1e-12 relative (the
tolerance of the single-instance tests)."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2411_06225_amd as rpr  # noqa: E402
from paper_2411_06225_amd import workloads as W  # noqa: E402


def burgers_instances(n, seed=5):
    rng = np.random.default_rng(seed)
    out = []
    for b in range(n):
        d = int(rng.choice([64, 96, 128, 200, 256]))
        # cell Reynolds number u dx / nu < 2 (central differences stay bounded)
        nu = float(10 ** rng.uniform(math.log10(2.0 / d), math.log10(2.0 / d) + 0.6))
        N = int(rng.integers(4, 9))
        tN = 1.0 + 0.2 * b
        Ts, dx, umax = tN / N, 2.0 / d, 2.0
        rho = 4 * nu / dx ** 2 + umax / dx               # spectral radius bound of the stencil
        nF = max(100, math.ceil(Ts * rho / 2.0))          # RK4 stable for dt * rho <= 2.78
        nG = max(8, math.ceil(Ts / (0.9 * min(dx ** 2 / (2 * nu), 2 * nu / umax ** 2))))  # forward Euler
        w = W.small(W.BURGERS_D128, nx=d, N=N, tN=tN, params=(nu,), F=(4, nF), G=(1, nG),
                    M=int(rng.integers(16, 48)), seed=100 + b)
        out.append(w)
    return out


def diffreact_instances():
    base = W.DIFFREACT_64
    return [W.small(base, nx=16, ny=16, N=6, tN=2.0, F=(4, 200), G=(1, 8), M=40, seed=21),
            W.small(base, nx=24, ny=20, N=8, tN=3.0, F=(4, 300), G=(1, 10), M=60, seed=22),
            W.small(base, nx=32, ny=32, N=5, tN=2.0, F=(4, 250), G=(1, 10), M=50, seed=23)]


def batch_problems(ws):
    problems = []
    for w in ws:
        A, z = W.random_weights(w)
        problems.append(dict(h=rpr.make_rhs(w.kind, w.nx, w.ny, w.domain, w.params), d=w.d, t0=w.t0, tN=w.tN,
                             N=w.N, F=w.F, G=w.G, M=w.M, activation=w.act, lam=w.lam, A=A, zeta=z))
    return problems


def execute_batch(plan, ws, scale=1.0):
    u0s = [scale * torch.tensor(W.initial_condition(w), dtype=torch.float64, device="cuda") for w in ws]
    outs = [torch.empty((w.N + 1, w.d), dtype=torch.float64, device="cuda") for w in ws]
    status = plan.execute(u0s, outs)
    torch.cuda.synchronize()
    infos = []
    for b in range(len(ws)):
        h = plan.instance(b)
        inf = h.info()
        inf["L_hist"], inf["chg_hist"] = h.history()
        infos.append(inf)
    return status, [o.cpu().numpy() for o in outs], infos


def run_batch(ws, precision=rpr.RPR_FP64, scale=1.0, **opt):
    plan = rpr.BatchPlan(batch_problems(ws), tol=[w.eps for w in ws], precision=precision, **opt)
    try:
        return execute_batch(plan, ws, scale)
    finally:
        plan.close()


def oracle_run(orc, w, k_max=None):
    pb = orc.problem(w.kind, w.nx, w.ny, w.domain, w.params)
    A, z = W.random_weights(w)
    return orc.parareal(pb, W.initial_condition(w), N=w.N, t0=w.t0, tN=w.tN, F=w.F, G=w.G, eps=w.eps,
                        net=orc.Net(A, z, w.act, w.lam, 0.0), nthreads=4, k_max=k_max)


@pytest.mark.parametrize("family", ["burgers", "diffreact"])
def test_batch_matches_oracle_per_instance(orc, family):
    ws = burgers_instances(10) if family == "burgers" else diffreact_instances()
    status, Us, infos = run_batch(ws)
    assert status == rpr.RPR_OK
    for w, Ug, ig in zip(ws, Us, infos):
        Uo, io = oracle_run(orc, w)
        assert ig["K"] == io["K"], w.name
        assert ig["L_hist"].tolist() == io["L_hist"].tolist()
        assert ig["rows_used"] == io["rows_used"]
        # identical non-finite pattern, finite entries within tolerance
        np.testing.assert_array_equal(np.isfinite(Ug), np.isfinite(Uo))
        fin = np.isfinite(Uo)
        err = np.abs(Ug[fin] - Uo[fin]).max() / np.abs(Uo[fin]).max()
        print(w.name, w.d, "K", ig["K"], "rel err %.2e" % err)
        assert err <= w.N * 1e-12


def test_batch_phase_times():
    # eager batches time their shared phases (every instance reports the
    # batch's); captured graphs have no events between the phases
    ws = burgers_instances(4)
    _, _, infos = run_batch(ws)
    for inf in infos:
        parts = inf["t_fine"] + inf["t_model"] + inf["t_sweep"]
        assert min(inf["t_fine"], inf["t_model"], inf["t_sweep"]) > 0.0
        assert 0.5 * inf["t_total"] <= parts <= inf["t_total"] * (1 + 1e-6)
        assert inf["t_fine"] == infos[0]["t_fine"]
    _, _, ginfos = run_batch(ws, graph=1)
    assert all(g["t_fine"] == g["t_model"] == g["t_sweep"] == -1.0 for g in ginfos)


def test_batch_of_one_equals_single_plan():
    w = burgers_instances(1)[0]
    _, Us, infos = run_batch([w])
    A, z = W.random_weights(w)
    U, info = rpr.solve(rpr.make_rhs(w.kind, w.nx, w.ny, w.domain, w.params),
                        torch.tensor(W.initial_condition(w), dtype=torch.float64, device="cuda"), t0=w.t0, tN=w.tN,
                        N=w.N, F=w.F, G=w.G, tol=w.eps, M=w.M, activation=w.act, lam=w.lam, A=A, zeta=z)
    assert infos[0]["K"] == info["K"]
    np.testing.assert_allclose(Us[0], U.cpu().numpy(), rtol=0, atol=w.N * 1e-12 * np.abs(Us[0]).max())


def test_mixed_precision_batch_close_to_fp64_serial_fine(orc):
    # E (mean over slices of the max error against the FP64 serial fine
    # solution) exceeds that of the FP64 iterate after as many iterations by
    # at most tau = 10 x E of the FP32 serial fine solution, instance by
    # instance
    from test_gpu_solve import E_err, gpu_serial_fine_fp32
    ws = burgers_instances(6, seed=9)
    status, Us, infos = run_batch(ws, precision=rpr.RPR_MIXED)
    for w, Ug, ig in zip(ws, Us, infos):
        assert ig["converged"] == 1
        pb = orc.problem(w.kind, w.nx, w.ny, w.domain, w.params)
        T = (w.tN - w.t0) / w.N
        Uf = orc.serial_fine(pb, w.F[0], w.F[1], T / w.F[1], w.N, W.initial_condition(w))
        Uo, _ = oracle_run(orc, w, k_max=ig["K"])
        tau = 10.0 * E_err(gpu_serial_fine_fp32(w), Uf)
        print(w.name, "mixed K", ig["K"], "E %.2e FP64 E %.2e tau %.2e" % (E_err(Ug, Uf), E_err(Uo, Uf), tau))
        assert E_err(Ug, Uf) <= E_err(Uo, Uf) + tau



def test_batch_graph_replays_match_plain_launches():
    """The captured iteration block (replayed poll_every iterations at a time;
    iterations after an instance stops return at once) gives the plain
    launches' results bit for bit, on repeated executes of one plan and after
    a change of input scale forces a new capture."""
    ws = burgers_instances(5, seed=13)
    plan = rpr.BatchPlan(batch_problems(ws), tol=[w.eps for w in ws], poll_every=3, graph=1)
    try:
        for scale in (1.0, 1.0, 0.45):  # 0.45 moves every instance's input scale s from 2 to 1
            _, Up, ip = run_batch(ws, poll_every=3, scale=scale)
            status, Ug, ig = execute_batch(plan, ws, scale)
            assert status == rpr.RPR_OK
            for b in range(len(ws)):
                assert ig[b]["K"] == ip[b]["K"] and ig[b]["input_scale"] == ip[b]["input_scale"], (scale, b)
                assert ig[b]["L_hist"].tolist() == ip[b]["L_hist"].tolist()
                np.testing.assert_array_equal(Ug[b], Up[b])
    finally:
        plan.close()


def test_nearest_neighbour_batch_matches_oracle_per_instance(orc):
    # every instance its own store and neighbour count; the chain of each
    # instance on one work-group.  Bound as for single plans: N 1e-12 plus the
    # forward error of the worst refit, 10 kappa 2^-53 (kappa from the
    # oracle's own neighbours).
    from test_gpu_solve import nn_refit_condition
    ws = burgers_instances(6, seed=9)
    ms = [2, 3, 4, 5, 8, 20]
    problems = batch_problems(ws)
    for q, m in zip(problems, ms):
        q["m_nn"] = m
    plan = rpr.BatchPlan(problems, tol=[w.eps for w in ws], correction=rpr.RPR_CORR_RANDNET_NN)
    try:
        status, Us, infos = execute_batch(plan, ws)
    finally:
        plan.close()
    assert status == rpr.RPR_OK
    for w, m, Ug, ig in zip(ws, ms, Us, infos):
        pb = orc.problem(w.kind, w.nx, w.ny, w.domain, w.params)
        A, z = W.random_weights(w)
        Uo, io = orc.parareal(pb, W.initial_condition(w), N=w.N, t0=w.t0, tN=w.tN, F=w.F, G=w.G, eps=w.eps,
                              corr=2, m_nn=m, net=orc.Net(A, z, w.act, w.lam, 0.0), nthreads=4, keep_iterates=True)
        assert ig["K"] == io["K"], w.name
        assert ig["L_hist"].tolist() == io["L_hist"].tolist()
        tol = max(w.N * 1e-12, 10 * nn_refit_condition(orc, w, io, m) * 2.0 ** -53)
        err = np.abs(Ug - Uo).max() / np.abs(Uo).max()
        print(w.name, w.d, "m", m, "K", ig["K"], "rel err %.2e tol %.1e" % (err, tol))
        assert err <= tol
