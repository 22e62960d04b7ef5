"""The per-entry parity check (CPU only): the oracle's entry scale S is the
MTTKRP of absolute values, and the check catches what a whole-matrix
Frobenius bound misses on a skewed tensor -- a light row that is dropped or
zeroed, one entry off by twice the tolerance -- while accepting the result
rounded to FP32."""

import numpy as np
import pytest

import oracle
from gpu_cases import assert_entrywise, case, entrywise_excess, factors_for, rel_fro, vals32
from synth import random_small_tensor


def brute_abs(dims, coords, vals, factors, mode):
    out = np.zeros((dims[mode], factors[0].shape[1]))
    for x in range(vals.shape[0]):
        t = np.abs(vals[x]) * np.ones(factors[0].shape[1])
        for m in range(len(dims)):
            if m != mode:
                t = t * np.abs(factors[m][coords[m, x]])
        out[coords[mode, x]] += t
    return out


def test_abs_scale_is_sum_of_absolute_terms():
    X = random_small_tensor((5, 4, 3, 2), 40, seed=3)
    rng = np.random.default_rng(4)
    facs = [rng.standard_normal((d, 3)) for d in X.dims]
    vals = rng.standard_normal(X.nnz)
    for n in range(X.nmodes):
        S = oracle.mttkrp_abs(X.dims, X.coords, vals, facs, n)
        np.testing.assert_allclose(S, brute_abs(X.dims, X.coords, vals, facs, n), rtol=1e-13, atol=0)
        M = oracle.mttkrp(X.dims, X.coords, vals, facs, n)
        assert np.all(np.abs(M) <= S * (1 + 1e-12))
        # sampled rows agree with the full scale
        rows = np.array([0, X.dims[n] - 1]) if X.dims[n] > 1 else np.array([0])
        np.testing.assert_allclose(oracle.mttkrp_abs(X.dims, X.coords, vals, facs, n, rows=rows), S[rows],
                                   rtol=1e-13, atol=0)


@pytest.fixture(scope="module")
def skewed():
    X = case("c2s")
    facs = [f.astype(np.float64) for f in factors_for(X, 16)]
    v = vals32(X).astype(np.float64)
    n = 2
    M = oracle.mttkrp(X.dims, X.coords, v, facs, n)
    S = oracle.mttkrp_abs(X.dims, X.coords, v, facs, n)
    return X, facs, v, n, M, S


def test_fp32_rounding_of_the_exact_result_passes(skewed):
    _, _, _, _, M, S = skewed
    assert_entrywise(M.astype(np.float32), M, S)


def test_zeroed_light_row_fails_entrywise_but_passes_frobenius(skewed):
    _, _, _, _, M, S = skewed
    nz = np.flatnonzero(np.abs(M).sum(axis=1) > 0)
    light = nz[np.argmin(np.abs(M[nz]).sum(axis=1))]
    bad = M.copy()
    bad[light] = 0.0
    assert rel_fro(bad, M) <= 1e-5  # invisible to the whole-matrix norm
    nbad, _ = entrywise_excess(bad, M, S)
    assert nbad == M.shape[1]


def test_dropped_nonzero_fails(skewed):
    """A mistake planted in the oracle's input: one nonzero of a light row
    left out of the sum."""
    X, facs, v, n, M, S = skewed
    counts = np.bincount(X.coords[n], minlength=X.dims[n])
    x = int(np.flatnonzero(counts[X.coords[n]] == 1)[0])
    keep = np.ones(X.nnz, dtype=bool)
    keep[x] = False
    got = oracle.mttkrp(X.dims, np.ascontiguousarray(X.coords[:, keep]), v[keep], facs, n)
    assert rel_fro(got, M) <= 1e-5
    with pytest.raises(AssertionError):
        assert_entrywise(got, M, S)


def test_one_entry_off_by_twice_the_tolerance_fails(skewed):
    _, _, _, _, M, S = skewed
    i, r = np.unravel_index(np.argmax(S), S.shape)
    bad = M.copy()
    bad[i, r] += 2e-5 * S[i, r]
    nbad, worst = entrywise_excess(bad, M, S)
    assert nbad == 1 and 1.9 < worst < 2.1
