"""The entry point that allocates nothing (rpr_randnet_features_noalloc):
through the C ABI it gives the results of rpr_randnet_features (the same
kernels; its split-K partial sums live in the library's per-device scratch),
on two calls in a row, the second with fewer rows, and rejects calls whose
partial sums would not fit the scratch."""
import ctypes as C

import numpy as np
import pytest

import paper_2411_06225_amd as rpr


def test_noalloc_rejects_oversized_calls_before_any_device_call():
    # d = 110592 takes 64 K splits: 64 x 256 x 300 doubles > 2^21
    L = rpr.lib()
    st = L.rpr_randnet_features_noalloc(300, 110592, 256, 1, 1.0, 1 << 20, 1 << 21, 1 << 22, 1 << 23, None)
    assert st == rpr.RPR_ERR_INVALID_ARG
    assert "scratch" in rpr.last_error()
    assert L.rpr_randnet_features_noalloc(4, 4, 0, 1, 1.0, 1, 2, 3, 4, None) == rpr.RPR_OK


@pytest.mark.gpu
def test_noalloc_features_equal_the_allocating_entry_point():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(11)
    M, d = 200, 8192
    A = torch.tensor(rng.uniform(-1, 1, (M, d)), device="cuda")
    z = torch.tensor(rng.uniform(-1, 1, M), device="cuda")
    for n, act in ((64, rpr.RPR_RELU), (13, rpr.RPR_TANH)):   # the second call smaller
        X = torch.tensor(rng.standard_normal((n, d)), device="cuda")
        want = torch.empty((n, M), dtype=torch.float64, device="cuda")
        got = torch.full((n, M), float("nan"), dtype=torch.float64, device="cuda")
        rpr.rpr_randnet_features(M, d, n, act, 4.0, A, z, X, want)
        rpr.rpr_randnet_features_noalloc(M, d, n, act, 4.0, A, z, X, got)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(got.cpu().numpy(), want.cpu().numpy())
