"""Pins of the oracle's MTTKRP and CP-ALS sweep against the dense definition
(explicit unfolding times explicit Khatri-Rao product), closed forms, special
cases and independent least-squares routines."""

import itertools

import numpy as np
import pytest

import oracle
from synth import make_config, make_factors, random_small_tensor
from test_oracle_encoding import example


def dense_of(dims, coords, vals):
    X = np.zeros(dims)
    np.add.at(X, tuple(coords), vals)
    return X


def unfold(X, n):
    """Mode-n matricization: rows i_n, columns the other modes in increasing
    order with the last one fastest."""
    return np.moveaxis(X, n, 0).reshape(X.shape[n], -1)


def khatri_rao(mats):
    """Column-wise Kronecker product A(1) (.) A(2) (.) ... in the given order."""
    R = mats[0].shape[1]
    cols = []
    for r in range(R):
        v = np.ones(1)
        for A in mats:
            v = np.kron(v, A[:, r])
        cols.append(v)
    return np.stack(cols, axis=1)


def brute_mttkrp(dims, coords, vals, factors, n):
    X = dense_of(dims, coords, vals)
    K = khatri_rao([factors[m] for m in range(len(dims)) if m != n])
    return unfold(X, n) @ K


def test_khatri_rao_helper_matches_definition():
    A = np.arange(6.0).reshape(3, 2)
    B = np.arange(8.0).reshape(4, 2) + 1
    K = khatri_rao([A, B])
    for i, j, r in itertools.product(range(3), range(4), range(2)):
        assert K[i * 4 + j, r] == A[i, r] * B[j, r]


@pytest.mark.parametrize("case", ["example", "small4", "c1"])
def test_mttkrp_equals_dense_unfolding(case):
    if case == "example":
        _, dims, coords, vals = example()
        R = 3
    elif case == "small4":
        X = random_small_tensor((5, 4, 3, 2), 40, seed=1)
        dims, coords, vals, R = X.dims, X.coords, X.vals, 4
    else:
        X = make_config("c1")
        dims, coords, vals, R = X.dims, X.coords, X.vals, 8
    factors = [np.random.default_rng(n).random((d, R)) for n, d in enumerate(dims)]
    for n in range(len(dims)):
        got = oracle.mttkrp(dims, coords, vals, factors, n)
        np.testing.assert_allclose(got, brute_mttkrp(dims, coords, vals, factors, n), rtol=1e-12, atol=1e-12)


def test_mttkrp_rank1_closed_form():
    rng = np.random.default_rng(4)
    dims = (30, 20, 10)
    a = []
    for d in dims:
        v = np.zeros(d)
        idx = rng.choice(d, 4, replace=False)
        v[idx] = rng.random(4) + 0.5
        a.append(v)
    cells = list(itertools.product(*[np.nonzero(v)[0] for v in a]))
    coords = np.array(cells, dtype=np.int64).T.copy()
    vals = np.array([a[0][i] * a[1][j] * a[2][k] for i, j, k in cells])
    R = 5
    factors = [rng.standard_normal((d, R)) for d in dims]
    for n in range(3):
        w = np.ones(R)
        for m in range(3):
            if m != n:
                w *= a[m] @ factors[m]
        np.testing.assert_allclose(oracle.mttkrp(dims, coords, vals, factors, n), np.outer(a[n], w), rtol=1e-12,
                                   atol=1e-13)


def test_mttkrp_single_nonzero():
    dims = (7, 9, 4, 3)
    coords = np.array([[5], [2], [3], [1]], dtype=np.int64)
    vals = np.array([2.5])
    R = 6
    factors = [np.random.default_rng(10 + n).random((d, R)) for n, d in enumerate(dims)]
    for n in range(4):
        got = oracle.mttkrp(dims, coords, vals, factors, n)
        expect = np.zeros((dims[n], R))
        row = 2.5 * np.ones(R)
        for m in range(4):
            if m != n:
                row = row * factors[m][coords[m, 0]]
        expect[coords[n, 0]] = row
        np.testing.assert_allclose(got, expect, rtol=1e-15)


def test_mttkrp_all_ones_factors_gives_slice_sums():
    X = random_small_tensor((11, 6, 9), 500, seed=2)
    R = 3
    ones = [np.ones((d, R)) for d in X.dims]
    for n in range(3):
        got = oracle.mttkrp(X.dims, X.coords, X.vals, ones, n)
        slice_sum = np.bincount(X.coords[n], weights=X.vals, minlength=X.dims[n])
        np.testing.assert_allclose(got, np.repeat(slice_sum[:, None], R, axis=1), rtol=1e-13)


def test_mttkrp_cross_mode_invariant():
    # sum_i M^(n)(i,r) A^(n)(i,r) = <X, a_r^(0) o ... o a_r^(N-1)> for every n
    X = random_small_tensor((8, 13, 5, 6), 700, seed=9)
    R = 4
    factors = [np.random.default_rng(30 + n).standard_normal((d, R)) for n, d in enumerate(X.dims)]
    inner = []
    for n in range(4):
        M = oracle.mttkrp(X.dims, X.coords, X.vals, factors, n)
        inner.append(np.sum(M * factors[n], axis=0))
    for n in range(1, 4):
        np.testing.assert_allclose(inner[n], inner[0], rtol=1e-12)


def test_mttkrp_duplicates_equal_summed_tensor():
    X = random_small_tensor((4, 3, 5), 300, seed=8)
    R = 2
    factors = [np.random.default_rng(n).random((d, R)) for n, d in enumerate(X.dims)]
    flat = np.ravel_multi_index(tuple(X.coords), X.dims)
    uniq, inv = np.unique(flat, return_inverse=True)
    summed = np.bincount(inv, weights=X.vals)
    ucoords = np.stack(np.unravel_index(uniq, X.dims)).astype(np.int64)
    assert len(uniq) < 300
    for n in range(3):
        np.testing.assert_allclose(oracle.mttkrp(X.dims, X.coords, X.vals, factors, n),
                                   oracle.mttkrp(X.dims, ucoords, summed, factors, n), rtol=1e-12)


def test_mttkrp_rows_matches_full():
    X = random_small_tensor((40, 30, 20), 2000, seed=5)
    R = 4
    factors = make_factors(X.dims, R, seed=5, dtype=np.float64)
    for n in range(3):
        full = oracle.mttkrp(X.dims, X.coords, X.vals, factors, n)
        rows = np.array([0, 3, 7, X.dims[n] - 1])
        np.testing.assert_array_equal(oracle.mttkrp_rows(X.dims, X.coords, X.vals, factors, n, rows), full[rows])


def test_mttkrp_empty_tensor_is_zero():
    dims = (3, 4, 5)
    coords = np.zeros((3, 0), dtype=np.int64)
    factors = [np.ones((d, 2)) for d in dims]
    assert not oracle.mttkrp(dims, coords, np.zeros(0), factors, 1).any()


# ---------------------------------------------------------------- CP-ALS sweep


def exact_low_rank(dims, R, seed, per_col=3):
    """X = sum_r lam_r a_r^(0) o ... o a_r^(N-1) with unit-norm columns whose
    supports are disjoint across r (so the sparse X lists every cell)."""
    rng = np.random.default_rng(seed)
    facs = []
    for d in dims:
        A = np.zeros((d, R))
        idx = rng.permutation(d)[: R * per_col].reshape(R, per_col)
        for r in range(R):
            A[idx[r], r] = rng.random(per_col) + 0.2
        A /= np.linalg.norm(A, axis=0)
        facs.append(A)
    lam = rng.random(R) + 1.0
    cells, vals = [], []
    for r in range(R):
        supp = [np.nonzero(A[:, r])[0] for A in facs]
        for c in itertools.product(*supp):
            v = lam[r]
            for A, i in zip(facs, c):
                v *= A[i, r]
            cells.append(c)
            vals.append(v)
    coords = np.array(cells, dtype=np.int64).T.copy()
    return facs, lam, coords, np.array(vals)


def test_als_sweep_fixed_point_of_exact_rank_r_tensor():
    dims = (20, 25, 30)
    facs, lam, coords, vals = exact_low_rank(dims, 4, seed=1)
    A, got_lam, ok = oracle.als_sweep(dims, coords, vals, facs)
    assert all(ok)
    for n in range(3):
        np.testing.assert_allclose(A[n], facs[n], atol=1e-12)
    np.testing.assert_allclose(got_lam, lam, rtol=1e-12)


def test_als_mode_update_equals_least_squares():
    # one mode update is argmin_A ||X_(n) - A K^T||_F; compare with lstsq on
    # the explicit unfolding and Khatri-Rao product
    X = random_small_tensor((6, 5, 4), 60, seed=21)
    R = 3
    facs = [np.random.default_rng(40 + n).random((d, R)) for n, d in enumerate(X.dims)]
    A, lam, ok, Ms = oracle.als_sweep(X.dims, X.coords, X.vals, facs, return_mttkrp=True)
    assert ok[0]
    K = khatri_rao([facs[1], facs[2]])
    sol, *_ = np.linalg.lstsq(K, unfold(dense_of(X.dims, X.coords, X.vals), 0).T, rcond=None)
    A0 = sol.T
    lam0 = np.linalg.norm(A0, axis=0)
    np.testing.assert_allclose(A[0], A0 / lam0, rtol=1e-9, atol=1e-12)
    for n in range(3):
        np.testing.assert_allclose(np.linalg.norm(A[n], axis=0), 1.0, rtol=1e-12)


def test_als_pseudoinverse_fallback_is_min_norm_least_squares():
    # two equal columns in every other factor make V singular: the update
    # must be the minimum-norm least-squares solution
    X = random_small_tensor((5, 6, 4), 50, seed=22)
    R = 3
    facs = [np.random.default_rng(50 + n).random((d, R)) for n, d in enumerate(X.dims)]
    for n in (1, 2):
        facs[n][:, 2] = facs[n][:, 1]
    A, lam, ok, Ms = oracle.als_sweep(X.dims, X.coords, X.vals, facs, return_mttkrp=True)
    assert not ok[0]
    K = khatri_rao([facs[1], facs[2]])
    sol = (np.linalg.pinv(K) @ unfold(dense_of(X.dims, X.coords, X.vals), 0).T).T
    lam0 = np.linalg.norm(sol, axis=0)
    np.testing.assert_allclose(A[0], sol / lam0, rtol=1e-7, atol=1e-9)


def test_parallel_cpu_baseline_equals_oracle():
    """The benchmark's parallel CPU leg computes the oracle's result."""
    X = make_config("c1")
    facs = make_factors(X.dims, 8, seed=2)
    for n in range(3):
        ref = oracle.mttkrp(X.dims, X.coords, X.vals, facs, n)
        got, used = oracle.mttkrp_parallel(X.dims, X.coords, X.vals, facs, n)
        assert used >= 1
        np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12)
