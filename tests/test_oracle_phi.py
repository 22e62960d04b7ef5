"""Pins of the oracle's CP-APR model update Phi and Pi rows (Algorithm
"alg:cp-apr-mu"): the dense matrix form (X_(n) ./ max(B Pi, eps)) Pi^T with
an explicit Khatri-Rao product on tiny tensors, the closed form when the
model matches the data at every nonzero, the eps floor, scaling in B, and
Pi rows equal to Khatri-Rao rows."""

import numpy as np

import oracle
from synth import random_small_tensor
from test_oracle_mttkrp import dense_of, khatri_rao, unfold


def dense_phi(dims, coords, vals, factors, B, n, eps):
    X = dense_of(dims, coords, vals)
    Xn = unfold(X, n)
    Pi = khatri_rao([factors[m] for m in range(len(dims)) if m != n]).T  # R x prod(other dims)
    model = B @ Pi
    Q = np.where(Xn != 0, Xn / np.maximum(model, eps), 0.0)
    return Q @ Pi.T


def test_phi_equals_dense_matrix_form():
    rng = np.random.default_rng(3)
    for dims, nnz, R in (((4, 5, 3), 25, 3), ((3, 4, 2, 5), 40, 4), ((6, 2, 3), 30, 2)):
        X = random_small_tensor(dims, nnz, seed=nnz)
        vals = rng.uniform(0.5, 2.0, X.nnz)
        facs = [rng.uniform(0.1, 1.0, (d, R)) for d in dims]
        for n in range(len(dims)):
            B = rng.uniform(0.1, 1.0, (dims[n], R))
            got = oracle.phi(dims, X.coords, vals, facs, B, n, 1e-10)
            np.testing.assert_allclose(got, dense_phi(dims, X.coords, vals, facs, B, n, 1e-10), rtol=1e-12,
                                       atol=1e-14)


def test_phi_when_the_model_matches_the_data():
    """If every nonzero equals the model B Pi there, the ratio is 1 and Phi is
    the MTTKRP of the tensor with unit values."""
    rng = np.random.default_rng(4)
    dims, R = (7, 6, 5), 3
    X = random_small_tensor(dims, 60, seed=2)
    facs = [rng.uniform(0.1, 1.0, (d, R)) for d in dims]
    for n in range(3):
        B = rng.uniform(0.1, 1.0, (dims[n], R))
        krp = oracle.pi_rows(dims, X.coords, facs, n)
        vals = np.sum(B[X.coords[n]] * krp, axis=1)
        got = oracle.phi(dims, X.coords, vals, facs, B, n, 1e-12)
        np.testing.assert_allclose(got, oracle.mttkrp(dims, X.coords, np.ones(X.nnz), facs, n), rtol=1e-12)


def test_phi_eps_floor_and_scaling_in_b():
    rng = np.random.default_rng(5)
    dims, R = (5, 4, 6), 4
    X = random_small_tensor(dims, 50, seed=3)
    vals = rng.uniform(1, 3, X.nnz)
    facs = [rng.uniform(0.1, 1.0, (d, R)) for d in dims]
    n, eps = 1, 1e-3
    # B = 0: every denominator is eps
    got = oracle.phi(dims, X.coords, vals, facs, np.zeros((dims[n], R)), n, eps)
    np.testing.assert_allclose(got, oracle.mttkrp(dims, X.coords, vals, facs, n) / eps, rtol=1e-12)
    # B scaled by c (no floor active): Phi scales by 1/c
    B = rng.uniform(0.5, 1.0, (dims[n], R))
    np.testing.assert_allclose(oracle.phi(dims, X.coords, vals, facs, 4.0 * B, n, 1e-12),
                               oracle.phi(dims, X.coords, vals, facs, B, n, 1e-12) / 4.0, rtol=1e-12)


def test_pi_rows_are_khatri_rao_rows():
    rng = np.random.default_rng(6)
    dims, R = (3, 4, 5), 2
    X = random_small_tensor(dims, 20, seed=4)
    facs = [rng.standard_normal((d, R)) for d in dims]
    for n in range(3):
        others = [m for m in range(3) if m != n]
        K = khatri_rao([facs[m] for m in others])  # rows: remaining modes row-major, last fastest
        idx = X.coords[others[0]] * dims[others[1]] + X.coords[others[1]]
        np.testing.assert_allclose(oracle.pi_rows(dims, X.coords, facs, n), K[idx], rtol=1e-14)
