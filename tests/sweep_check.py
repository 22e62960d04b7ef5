"""Per-mode parity of a CP-ALS sweep with the FP64 oracle (test helper).

A sweep updates the modes in order, so mode n's update used the new factors
of modes < n and the starting factors of modes > n.  For every mode the
oracle recomputes that update (Algorithm "alg:cp-als": V from the Grams,
M = MTTKRP, A = M V^+, column norms) from exactly those factors and checks:

* the normal-equation residual of the GPU's normalized factor with the best
  column scales, min_D ||A D V - M||_F / ||M||_F, within 1e-5 (the MTTKRP
  bound) plus u * cond(V) for the FP32 storage of A (u = 2^-24): a bound free
  of the solve's conditioning apart from that storage term;
* the forward error of the factor (columns weighted by lambda) within
  max(1e-5, cond(V) * 1e-5), the MTTKRP bound amplified by the solve;
* unit column norms, and lambda of the last mode.
"""

from __future__ import annotations

import numpy as np

import oracle
from gpu_cases import bf16_round, rel_fro, say

U32 = 2.0 ** -24


def mode_update(dims, coords, vals, cur, n, quantize=False):
    """Oracle update of mode n from the factors the GPU held at that point
    (Grams from the FP32 masters; MTTKRP from BF16-rounded factors when
    ``quantize``).  Returns (A normalized, lambda, cholesky ok, V, M)."""
    v = np.asarray(vals, dtype=np.float64)
    f64 = [np.asarray(c, dtype=np.float64) for c in cur]
    fm = [bf16_round(c).astype(np.float64) for c in cur] if quantize else f64
    R = cur[0].shape[1]
    V = np.ones((R, R))
    for m in range(len(dims)):
        if m != n:
            V *= f64[m].T @ f64[m]
    M = oracle.mttkrp(dims, coords, v, fm, n)
    An, ok = oracle._solve_spd_or_pinv(V, M)
    lam = np.linalg.norm(An, axis=0)
    return An / np.where(lam > 0, lam, 1.0), lam, ok, V, M


def scaled_residual(A, V, M):
    """min over diagonal D of ||A D V - M||_F / ||M||_F.  With
    C_s = A(:, s) V(s, :), the normal equations are G d = b with
    G_st = <A_s, A_t> <V_s, V_t> and b_s = <A_s, M V_s^T>."""
    A = np.asarray(A, dtype=np.float64)
    G = (A.T @ A) * (V @ V.T)
    b = np.einsum("is,ir,sr->s", A, M, V)
    d = np.linalg.lstsq(G, b, rcond=None)[0]
    return rel_fro((A * d) @ V, M), d


def check_sweep(dims, coords, vals, start, new, lam_last, what="", quantize=False, expect_chol=True):
    """Check every mode of one sweep from ``start`` that produced ``new``
    (lists of FP32 arrays) and lambda ``lam_last`` of the last mode."""
    N = len(dims)
    worst = 0.0
    for n in range(N):
        cur = [new[m] if m < n else start[m] for m in range(N)]
        ref, ref_lam, ok, V, M = mode_update(dims, coords, vals, cur, n, quantize)
        if expect_chol:
            assert ok, (what, n)
        kappa = np.linalg.cond(V)
        res, _ = scaled_residual(new[n], V, M)
        res_tol = 1e-5 + U32 * kappa
        e = rel_fro(np.asarray(new[n], dtype=np.float64) * ref_lam, ref * ref_lam)
        fwd_tol = max(1e-5, kappa * 1e-5)
        say(f"    {what} mode {n}: residual {res:.2e} (tol {res_tol:.1e})  factor err {e:.2e} "
            f"(tol {fwd_tol:.1e}) cond(V) {kappa:.1f}")
        assert res <= res_tol, (what, n, res)
        assert e <= fwd_tol, (what, n, e)
        nz = ref_lam > 0
        np.testing.assert_allclose(np.linalg.norm(np.asarray(new[n], dtype=np.float64)[:, nz], axis=0), 1.0,
                                   rtol=1e-5)
        if n == N - 1:
            assert rel_fro(np.asarray(lam_last), ref_lam) <= fwd_tol
            # with the GPU's own lambda the residual is bounded the same way
            res_l = rel_fro(np.asarray(new[n], dtype=np.float64) * np.asarray(lam_last) @ V, M)
            assert res_l <= res_tol, (what, n, res_l)
        worst = max(worst, res)
    return worst
