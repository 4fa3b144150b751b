"""Writes full-size oracle runs of RandNet-Parareal for the GPU tests:

  diffreact_64x64_oracle.json   64 x 64 diffusion-reaction (N = 64 slices, RK4 x
                                4000 fine steps, RK1 x 10 coarse steps, 200 ReLU
                                neurons, lambda = eps = 1e-6); about a minute
  swe_192x192_oracle.json       192 x 192 shallow water (N = 256 slices, RK4 x
                                1000 fine steps, RK1 x 8 coarse steps, 300 ReLU
                                neurons, lambda = eps = 1e-6); about 45 minutes
                                on 8 threads, the serial fine solution on one of
                                them beside the parareal run

Calls only oracle/ and the seeded input generators.  Each fixture keeps the
iteration count, the L and change histories, the accuracy E against the
oracle's serial fine solution, a fixed sample of U^K entries and of the serial
fine solution (every slot, the same seeded positions per slot), and the
condition number kappa_2(Phi^T Phi + lambda I) of the ridge system fitted at
each iteration (from the oracle's own pairs: inputs U_{i-1}^{k-1},
i = L_{k-1}+1..N), so the GPU tests can compare at full size, with the bound
the ridge solves imply, without re-running the oracle.

    python tests/golden/make_oracle_reference.py [nthreads] [diffreact|swe]
"""
import json
import os
import sys
import threading

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2411_06225_amd import workloads as W  # noqa: E402

# workload, output file, sampled positions per slot, iterates kept (the run
# must converge before), description
CASES = {
    "diffreact": (W.DIFFREACT_64, "diffreact_64x64_oracle.json", 32, 64,
                  "oracle RandNet-Parareal run of the 64x64 diffusion-reaction workload"),
    "swe": (W.SWE_192, "swe_192x192_oracle.json", 16, 8,
            "oracle RandNet-Parareal run (FP64) of the 192x192 shallow-water workload, N = 256"),
}


def ridge_condition_numbers(w, net, info):
    """kappa_2(Phi^T Phi + lambda I) of the readout fitted at each iteration k:
    Phi holds the features of every pair input so far, U_{i-1}^{j-1} for
    i = L_{j-1}+1..N and j = 1..k (eq. "ridgeless"; Alg. "RandNets training
    procedure")."""
    rows, kappas = [], []
    for k in range(1, info["K"] + 1):
        L = int(info["L_hist"][k - 1])
        rows.append(oracle.features(net, info["U_iter"][k - 1][L:w.N]))
        Phi = np.concatenate(rows)
        kappas.append(float(np.linalg.cond(Phi.T @ Phi + w.lam * np.eye(w.M))))
    return kappas


def main():
    nthreads = int(sys.argv[1]) if len(sys.argv) > 1 else 8
    case = sys.argv[2] if len(sys.argv) > 2 else "diffreact"
    w, fname, n_sample, k_max, what = CASES[case]
    pb = oracle.problem(w.kind, w.nx, w.ny, w.domain, w.params)
    u0 = W.initial_condition(w)
    A, zeta = W.random_weights(w)
    net = oracle.Net(A, zeta, w.act, w.lam, 0.0)
    T = (w.tN - w.t0) / w.N
    # the serial fine solution is one slot after another on one thread; it
    # runs beside the parareal run (ctypes releases the interpreter lock)
    fine = {}
    th = threading.Thread(target=lambda: fine.update(U=oracle.serial_fine(pb, w.F[0], w.F[1], T / w.F[1], w.N, u0)))
    th.start()
    U, info = oracle.parareal(pb, u0, N=w.N, t0=w.t0, tN=w.tN, F=w.F, G=w.G, eps=w.eps, net=net,
                              k_max=k_max, nthreads=max(nthreads - 1, 1), keep_iterates=True)
    th.join()
    assert info["converged"], "the run must stop by the rule before the iterates kept run out"
    kappas = ridge_condition_numbers(w, oracle.Net(A, zeta, w.act, w.lam, oracle.input_scale(u0)), info)
    Uf = fine["U"]
    E = float(np.mean(np.abs(U[1:] - Uf[1:]).max(axis=1)))
    rng = np.random.default_rng(2024)
    idx = rng.choice(w.d, n_sample, replace=False)
    out = {
        "what": what,
        "workload": w.name,
        "K": info["K"],
        "L_hist": info["L_hist"].tolist(),
        "chg_hist": info["chg_hist"].tolist(),
        "rows_used": info["rows_used"],
        "E_vs_serial_fine": E,
        "sample_index": idx.tolist(),
        "U_sample": U[:, idx].tolist(),
        "U_absmax": float(np.abs(U).max()),
        "serial_fine_sample": Uf[:, idx].tolist(),
        "ridge_kappa": kappas,
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), fname)
    with open(path, "w") as f:
        json.dump(out, f)
    print("wrote", path, "K", info["K"], "E", E, "kappa", ["%.2e" % x for x in kappas])


if __name__ == "__main__":
    main()
