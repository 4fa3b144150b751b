"""The stored full-size oracle runs (tests/golden/*_oracle.json) against
properties the method fixes, so that a fixture the GPU tests compare with is
itself checked:

- slot 0 is u0 (Alg. "Parareal (generic)": U_0^k = u0);
- Parareal's exactness: while the converged-slot counter advances by exactly
  one per iteration (L_j = j for j <= p), iteration j fine-solves slot j from
  an exact state, so slots 1 .. p + 1 equal the serial fine solution bit for
  bit (same F, same arithmetic); the slot after them carries a prediction;
- the run stopped by the rule: L is non-decreasing and ends at N, with K + 1
  entries, and the last change is below the tolerance;
- the stored accuracy E (mean over slots of the max error against the serial
  fine solution, over all entries) bounds the same measure on the sample.
"""
import json
import os

import numpy as np
import pytest

from paper_2411_06225_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
FIXTURES = [("diffreact_64x64_oracle.json", W.DIFFREACT_64), ("swe_192x192_oracle.json", W.SWE_192)]


@pytest.mark.parametrize("fname,w", FIXTURES, ids=[f[0] for f in FIXTURES])
def test_stored_oracle_run_satisfies_parareal_invariants(fname, w):
    g = json.load(open(os.path.join(GOLDEN, fname)))
    U, S = np.asarray(g["U_sample"]), np.asarray(g["serial_fine_sample"])
    idx = np.asarray(g["sample_index"])
    assert g["workload"] == w.name and U.shape == S.shape == (w.N + 1, idx.size)
    np.testing.assert_array_equal(U[0], W.initial_condition(w)[idx])
    np.testing.assert_array_equal(S[0], W.initial_condition(w)[idx])
    L, K = g["L_hist"], g["K"]
    assert len(L) == K + 1 and L[0] == 0 and L[-1] == w.N
    assert all(a <= b for a, b in zip(L, L[1:]))
    assert g["chg_hist"][-1] <= w.eps
    p = 0
    while p + 1 < len(L) and L[p + 1] == p + 1:
        p += 1
    for i in range(1, min(p + 1, w.N) + 1):
        np.testing.assert_array_equal(U[i], S[i])
    E_sample = float(np.mean(np.abs(U[1:] - S[1:]).max(axis=1)))
    assert 0.0 < E_sample <= g["E_vs_serial_fine"]
    assert len(g["ridge_kappa"]) == K and all(k >= 1.0 for k in g["ridge_kappa"])
