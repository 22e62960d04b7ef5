"""Pins of the oracle's CP fit and CP-ALS loop (Algorithm "alg:cp-als":
sweeps repeat until the fit ceases to improve): the fit equals the one from
an explicit dense reconstruction, is 1 for an exact model and 0 for the
empty model, and ALS sweeps never lower it."""

import numpy as np

import oracle
from synth import random_small_tensor
from test_oracle_mttkrp import dense_of, exact_low_rank


def dense_model(dims, factors, lam):
    out = np.zeros(dims)
    for r in range(len(lam)):
        t = np.array(lam[r])
        for f in factors:
            t = np.multiply.outer(t, f[:, r])
        out += t
    return out


def test_norm_sums_duplicates_first():
    coords = np.array([[0, 1, 0, 0], [2, 0, 2, 2]], dtype=np.int64)
    vals = np.array([1.0, 5.0, 2.0, -4.0])
    # cell (0, 2) holds 1 + 2 - 4 = -1, cell (1, 0) holds 5
    assert oracle.tensor_norm2((2, 3), coords, vals) == 26.0
    assert oracle.tensor_norm2((2, 3), coords[:, :0], vals[:0]) == 0.0


def test_fit_equals_dense_reconstruction():
    rng = np.random.default_rng(5)
    for dims, nnz, R in (((4, 5, 3), 30, 3), ((3, 4, 2, 5), 50, 4), ((6, 2, 3), 80, 2)):
        X = random_small_tensor(dims, nnz, seed=nnz)  # may repeat coordinates
        vals = rng.standard_normal(X.nnz)
        facs = [rng.standard_normal((d, R)) for d in dims]
        lam = rng.uniform(0.5, 2.0, R)
        Xd = dense_of(dims, X.coords, vals)
        want = 1.0 - np.linalg.norm(Xd - dense_model(dims, facs, lam)) / np.linalg.norm(Xd)
        got = oracle.cp_fit(dims, X.coords, vals, facs, lam)
        assert abs(got - want) <= 1e-12, (got, want)


def test_fit_of_exact_model_is_one_and_of_zero_model_is_zero():
    dims = (30, 20, 15)
    facs, lam, coords, vals = exact_low_rank(dims, 4, seed=2)
    assert oracle.cp_fit(dims, coords, vals, facs, lam) >= 1.0 - 1e-6
    assert oracle.cp_fit(dims, coords, vals, facs, np.zeros_like(lam)) == 0.0


def test_cp_als_fit_never_decreases_and_stops_at_tolerance():
    X = random_small_tensor((12, 10, 8), 300, seed=9)
    vals = np.random.default_rng(1).uniform(0, 1, X.nnz)
    facs = [np.random.default_rng(2 + m).uniform(0, 1, (d, 3)) for m, d in enumerate(X.dims)]
    _, _, fits = oracle.cp_als(X.dims, X.coords, vals, facs, max_sweeps=40, tol=1e-6)
    assert len(fits) >= 2
    assert np.all(np.diff(fits) >= -1e-12)
    if len(fits) < 40:
        assert abs(fits[-1] - fits[-2]) < 1e-6
        assert all(abs(b - a) >= 1e-6 for a, b in zip(fits[:-2], fits[1:-1]))


def test_cp_als_recovers_an_exact_low_rank_tensor():
    dims = (20, 15, 12)
    facs, _, coords, vals = exact_low_rank(dims, 3, seed=4)
    rng = np.random.default_rng(3)
    start = [f + 0.05 * rng.standard_normal(f.shape) for f in facs]
    _, _, fits = oracle.cp_als(dims, coords, vals, start, max_sweeps=50, tol=1e-10)
    assert fits[-1] >= 1.0 - 1e-6
