"""Pins of the oracle's CP-APR driver (Algorithm "alg:cp-apr-mu",
multiplicative updates): the exact fixed point of a model with disjoint
column supports (Phi = 1 on the support, converged at the first inner
iteration, lambda = column sums), the monotone decrease of the Poisson
objective that multiplicative updates guarantee, column-stochastic factors,
and the inadmissible-zero adjustment S releasing a factor entry stuck at 0."""

import numpy as np
import pytest

import oracle
from synth import random_small_tensor


def block_model(seed=0):
    """Rank-3 model with disjoint supports per component: column r of every
    factor is nonzero only on its own block of indices and sums to 1.  The
    tensor holds every cell of each component's block with the model value
    there, so the model equals the data on the support and is 0 elsewhere."""
    rng = np.random.default_rng(seed)
    blocks = [((0, 2), (0, 3), (0, 2)), ((2, 5), (3, 5), (2, 3)), ((5, 6), (5, 8), (3, 6))]
    dims = (6, 8, 6)
    R = len(blocks)
    facs = [np.zeros((d, R)) for d in dims]
    for r, blk in enumerate(blocks):
        for m, (a, b) in enumerate(blk):
            w = rng.uniform(0.5, 1.5, b - a)
            facs[m][a:b, r] = w / w.sum()
    lam = np.array([20.0, 7.0, 13.0])
    coords, vals = [], []
    for r, blk in enumerate(blocks):
        for i in range(*blk[0]):
            for j in range(*blk[1]):
                for k in range(*blk[2]):
                    coords.append((i, j, k))
                    vals.append(lam[r] * facs[0][i, r] * facs[1][j, r] * facs[2][k, r])
    return dims, np.ascontiguousarray(np.array(coords, dtype=np.int64).T), np.array(vals), facs, lam


def test_fixed_point_of_an_exact_model():
    dims, coords, vals, facs, lam = block_model()
    A, lam2, k, inner, conv = oracle.cp_apr_mu(dims, coords, vals, facs, lam=lam, k_max=5, l_max=10, tau=1e-8)
    assert conv and k == 1 and inner == [[1, 1, 1]]
    for a, f in zip(A, facs):
        np.testing.assert_allclose(a, f, rtol=0, atol=1e-12)
    np.testing.assert_allclose(lam2, lam, rtol=1e-12)
    # and Phi is exactly 1 on the support there
    B = facs[0] * lam[None, :]
    P = oracle.phi(dims, coords, vals, facs, B, 0, 1e-10)
    np.testing.assert_allclose(P[B > 0], 1.0, rtol=1e-12)


@pytest.mark.parametrize("dims,nnz,R", [((7, 6, 5), 60, 3), ((5, 4, 6, 3), 90, 4)])
def test_objective_never_increases(dims, nnz, R):
    X = random_small_tensor(dims, nnz, seed=nnz)
    rng = np.random.default_rng(R)
    vals = rng.poisson(3.0, X.nnz) + 1.0
    A = [rng.uniform(0.1, 1.0, (d, R)) for d in dims]
    lam = np.ones(R)
    f_prev = oracle.poisson_objective(dims, X.coords, vals, A, lam)
    for _ in range(6):
        A, lam, k, inner, conv = oracle.cp_apr_mu(dims, X.coords, vals, A, lam=lam, k_max=1, l_max=3, tau=1e-12)
        f = oracle.poisson_objective(dims, X.coords, vals, A, lam)
        assert f <= f_prev + 1e-10 * abs(f_prev), (f, f_prev)
        f_prev = f
        for a in A:  # lambda carries the scale: factor columns sum to 1
            np.testing.assert_allclose(a.sum(axis=0), 1.0, rtol=1e-12)


def test_inadmissible_zero_is_released_by_s():
    """A factor entry at exactly 0 that the data wants positive (Phi > 1
    there) stays 0 under pure multiplicative updates; S adds kappa in the
    next outer iteration and the entry becomes positive."""
    dims, coords, vals, facs, lam = block_model(seed=1)
    start = [f + 0.05 for f in facs]  # a full-support start ...
    start[1][3, 1] = 0.0  # ... with one entry inside component 1's block at 0
    for f in start:
        f /= f.sum(axis=0, keepdims=True)
    A0, _, _, _, _ = oracle.cp_apr_mu(dims, coords, vals, start, k_max=2, l_max=5, tau=1e-12, kappa=0.0)
    A1, _, _, _, _ = oracle.cp_apr_mu(dims, coords, vals, start, k_max=2, l_max=5, tau=1e-12, kappa=1e-2,
                                      kappa_tol=1e-10)
    assert A0[1][3, 1] == 0.0
    assert A1[1][3, 1] > 0.0
