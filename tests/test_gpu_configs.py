"""GPU solves at the sizes of the workloads the other tests reduce: the batch
of uneven 1D Burgers problems with d up to 4096 (the persistent fine-solve
launch's longest strips, the one-work-group chains), tiled solves on
wall-bounded grids of several tiles in both directions, and the full
128 x 128 Brusselator and 192 x 192 shallow-water grids with a few steps.
Step counts and time spans are reduced so the oracle finishes; grids, sizes
and parameter ranges are the workloads' own."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2411_06225_amd as rpr  # noqa: E402
from paper_2411_06225_amd import workloads as W  # noqa: E402
from test_gpu_batch import batch_problems, execute_batch, run_batch  # noqa: E402
from test_gpu_solve import E_err, assert_same_run, gpu_solve, gpu_serial_fine_fp32, orc_solve, tiled  # noqa: E402


def config4_instances(ds=(256, 512, 1024, 2048, 4096, 4096, 1024, 256), N=8, tN=0.02, seed=4):
    """Burgers problems of the batched workload (periodic [-1, 1], d from
    {256, ..., 4096}, nu log-uniform in [1e-3, 1e-1], sines initial state,
    100 tanh neurons) with N = 8 slices of a short span; steps per slice by
    the workload's rule (RK4: dt rho <= 2.5, forward Euler: dt <= 0.9 dx^2 /
    (2 nu) and <= 0.9 * 2 nu / u_max^2) with lower floors."""
    rng = np.random.default_rng(seed)
    nus = 10.0 ** rng.uniform(-3.0, -1.0, len(ds))
    out = []
    Ts = tN / N
    for b, (d, nu) in enumerate(zip(ds, nus)):
        dx, umax = 2.0 / d, 2.0
        rho = 4 * nu / dx ** 2 + umax / dx
        nf = max(50, math.ceil(Ts * rho / 2.5))
        ng = max(4, math.ceil(Ts / min(0.9 * dx ** 2 / (2 * nu), 0.9 * 2 * nu / umax ** 2)))
        out.append(W.Workload(f"burgers_c4_{b}", W.BURGERS1D, int(d), 1, (-1.0, 1.0, -1.0, 1.0), (float(nu),), N,
                              0.0, tN, (W.RK4, nf), (W.RK1, ng), 100, W.TANH, 1e-6, 1e-6, "burgers_sines", 2000 + b))
    return out


def oracle_run(orc, w, k_max=None):
    pb = orc.problem(w.kind, w.nx, w.ny, w.domain, w.params)
    A, z = W.random_weights(w)
    return orc.parareal(pb, W.initial_condition(w), N=w.N, t0=w.t0, tN=w.tN, F=w.F, G=w.G, eps=w.eps,
                        net=orc.Net(A, z, w.act, w.lam, 0.0), nthreads=8, k_max=k_max)


def _oracle_module():
    import oracle
    return oracle


def oracle_serial_fine(orc, w):
    pb = orc.problem(w.kind, w.nx, w.ny, w.domain, w.params)
    T = (w.tN - w.t0) / w.N
    return orc.serial_fine(pb, w.F[0], w.F[1], T / w.F[1], w.N, W.initial_condition(w))


@pytest.fixture(scope="module")
def c4(orc):
    ws = config4_instances()
    runs = [oracle_run(orc, w) for w in ws]
    fine = [oracle_serial_fine(orc, w) for w in ws]
    return ws, runs, fine


def test_batch_at_workload_sizes_matches_oracle_per_instance(c4):
    ws, runs, _ = c4
    status, Us, infos = run_batch(ws)
    assert status == rpr.RPR_OK
    for w, Ug, ig, (Uo, io) in zip(ws, Us, infos, runs):
        print(w.name, "d", w.d, "nu %.2e" % w.params[0], "F", w.F, "G", w.G, "K", ig["K"])
        assert_same_run(Ug, ig, Uo, io, w.N)


def test_autotuned_batch_at_workload_sizes_matches_oracle_per_instance(c4, tmp_path, monkeypatch):
    # the batch autotuner picks the persistent launch's work-group count by
    # timing it; the items are independent, so the values are those of the
    # untuned batch bit for bit, and the choice lands in the tuning table
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("RPR_TUNE_CACHE", str(cache))
    ws, runs, _ = c4
    status, Us, infos = run_batch(ws, autotune=1)
    assert status == rpr.RPR_OK
    _, Up, _ = run_batch(ws)
    for w, Ug, ig, Ub, (Uo, io) in zip(ws, Us, infos, Up, runs):
        assert_same_run(Ug, ig, Uo, io, w.N)
        np.testing.assert_array_equal(Ug, Ub)
    text = cache.read_text() if cache.exists() else ""
    print(text[:400])


def test_reduced_precision_batch_at_workload_sizes_within_tau(c4):
    # every instance: E of the reduced-precision solve against the FP64
    # serial fine solution exceeds that of the FP64 iterate after as many
    # iterations by at most tau = 10 x E of the FP32 serial fine solution
    ws, runs, fine = c4
    status, Us, infos = run_batch(ws, precision=rpr.RPR_MIXED)
    for w, Ug, ig, Uf in zip(ws, Us, infos, fine):
        assert ig["converged"] == 1
        Uo, io = oracle_run(_oracle_module(), w, k_max=ig["K"])
        tau = 10.0 * E_err(gpu_serial_fine_fp32(w), Uf)
        print(w.name, "mixed K", ig["K"], "E %.2e" % E_err(Ug, Uf), "FP64 E %.2e" % E_err(Uo, Uf), "tau %.2e" % tau)
        assert E_err(Ug, Uf) <= E_err(Uo, Uf) + tau


def test_batch_at_workload_sizes_graph_equals_plain_launches(c4):
    ws, _, _ = c4
    _, Up, ip = run_batch(ws, precision=rpr.RPR_MIXED)
    _, Ug, ig = run_batch(ws, precision=rpr.RPR_MIXED, graph=1)
    for b in range(len(ws)):
        assert ig[b]["K"] == ip[b]["K"]
        np.testing.assert_array_equal(Ug[b], Up[b])


# ---- tiled solves on wall-bounded grids of several tiles each way ----
DR_WIDE = W.small(W.DIFFREACT_64, nx=130, ny=40, N=8, tN=2.0, F=(4, 40), G=(1, 20), M=40)
SWE_WIDE = W.small(W.SWE_192, nx=130, ny=40, N=8, tN=0.2, F=(4, 40), G=(1, 20), M=40, precision="fp64")


@pytest.mark.parametrize("name,w", [("diffreact_130x40", DR_WIDE), ("swe_130x40", SWE_WIDE)])
def test_tiled_walls_several_tiles_match_oracle(orc, name, w):
    # 130 x 40 cells: 3 x 3 tiles of 64 x 16 (one pass per stage) or 3 x 2
    # of 64 x 32 (one pass per RK4 step), ragged at the east and north walls;
    # the coarse solver runs forward Euler in passes of 8 steps per tile
    wt = tiled(w)
    Ug, ig = gpu_solve(wt)
    Uo, io = orc_solve(orc, w)
    assert_same_run(Ug, ig, Uo, io, w.N)


@pytest.mark.parametrize("name,w", [("diffreact_130x40", DR_WIDE), ("swe_130x40", SWE_WIDE)])
def test_tiled_reduced_precision_coarse_passes_do_not_depend_on_schedule(name, w):
    # Reduced precision, classical correction (no hidden layer, whose partial
    # sums follow the chain's grid): the multi-step coarse solver's tiles
    # read their halo's state and compensation from the previous pass only,
    # so any number of work-groups sharing the tiles (one: the tiles one
    # after the other) and the captured graph's segment kernels reproduce the
    # plain launch bit for bit
    wt = tiled(w)
    Ue, ie = gpu_solve(wt, prec=rpr.RPR_MIXED, corr=rpr.RPR_CORR_PARAREAL)
    for wgs in (1, 7, 33):
        Uw, iw = gpu_solve(wt, prec=rpr.RPR_MIXED, corr=rpr.RPR_CORR_PARAREAL, chain_wgs=wgs)
        assert iw["K"] == ie["K"], wgs
        np.testing.assert_array_equal(Uw, Ue)
    Ug, ig = gpu_solve(wt, prec=rpr.RPR_MIXED, corr=rpr.RPR_CORR_PARAREAL, graph=1, chain_wgs=5)
    assert ig["K"] == ie["K"]
    np.testing.assert_array_equal(Ug, Ue)


# ---- the full grids with a few steps ----
# (step counts inside both solvers' stability regions: the pre-check's
# ratios are 0.62 / 0.86 and 0.23 / 0.79)
BRUSS_FULL = W.BRUSS_128.replace(name="bruss_128x128_n4", N=4, tN=0.4, F=(4, 40), G=(1, 40), precision="fp64")
SWE_FULL = W.SWE_192.replace(name="swe_192x192_n4", N=4, tN=0.02, F=(4, 20), G=(1, 8), precision="fp64")


@pytest.mark.parametrize("name,w", [("bruss_128x128", BRUSS_FULL), ("swe_192x192", SWE_FULL)])
def test_full_grid_solve_matches_oracle(orc, name, w):
    # With N = 4 the ridge matrices hold 4 .. 16 pairs for 100 / 300 neurons:
    # nearly singular (lambda = 1e-6), so the bound adds the Cholesky solve's
    # forward-error bound 10 kappa 2^-53 (kappa from the oracle's own pairs), as
    # the iterate-by-iterate test does
    from test_gpu_solve import ridge_condition_numbers
    Ug, ig = gpu_solve(w, stability=1)
    assert ig["unstable"] == 0 and ig["stab_F"] < 1 and ig["stab_G"] < 1
    Uo, io = orc_solve(orc, w, keep=True)
    assert ig["K"] == io["K"] and ig["L_hist"].tolist() == io["L_hist"].tolist()
    assert ig["rows_used"] == io["rows_used"]
    tol = max(w.N * 1e-12, 10 * max(ridge_condition_numbers(orc, w, io)) * 2.0 ** -53)
    err = np.abs(Ug - Uo).max() / np.abs(Uo).max()
    print(name, "K", ig["K"], "rel err %.2e tol %.1e" % (err, tol))
    assert err <= tol
