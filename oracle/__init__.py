"""FP64 CPU oracle for ALTO MTTKRP and the CP-ALS sweep -- TEST INFRASTRUCTURE.

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never does; it shares
no code with this package (see ``alto_oracle.c`` for the per-nonzero loops).

The per-nonzero loops (encode, decode, order, partition, MTTKRP) are plain C
in ``alto_oracle.c``; the CP-ALS sweep is composed here in NumPy FP64 from
those loops and library primitives (matrix products, Cholesky, symmetric
eigendecomposition), step by step as Algorithm "alg:cp-als" of the paper
(arXiv 2403.06348, Sec. "CP-ALS") lists them.

Parity is pinned (in ``tests/test_oracle_*.py``) against: the paper's worked
example (Fig. "format-comparison"(a), Sec. "ALTO Tensor Generation" and
"Workload Partitioning and Scheduling"), Eq. 1-3, dense-unfolding brute
force, the rank-1 closed form, single-nonzero and all-ones special cases,
the cross-mode invariant, a NumPy stable sort, and the exact CP-ALS fixed
point of an exactly low-rank tensor.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "alto_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

MAX_MODES = 16


_PAR_SRC = os.path.join(_HERE, "cpu_parallel.c")
_PAR_LIB = os.path.join(_HERE, "libcpu_parallel.so")
_par = None


def build_oracle(force: bool = True) -> str:
    """Compile the C oracle (and the parallel CPU baseline) with gcc (host only)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    if force or not os.path.exists(_PAR_LIB):
        tmp = _PAR_LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-fopenmp", "-shared", "-fPIC", "-o", tmp,
                               _PAR_SRC])
        os.replace(tmp, _PAR_LIB)
    return _LIB


def _P():
    global _par
    if _par is None:
        if not os.path.exists(_PAR_LIB):
            build_oracle(force=True)
        lib = ctypes.CDLL(_PAR_LIB)
        P = ctypes.c_void_p
        lib.par_mttkrp.argtypes = [ctypes.c_int, P, ctypes.c_int64, P, P, ctypes.c_int, P, ctypes.c_int, P]
        lib.par_mttkrp.restype = ctypes.c_int
        lib.par_threads.restype = ctypes.c_int
        _par = lib
    return _par


def mttkrp_parallel(dims, coords, vals, factors, mode: int):
    """The parallel CPU baseline (OpenMP over nonzeros, private outputs, in
    cpu_parallel.c): (output, threads used).  Not part of the checked oracle."""
    d = _dims(dims)
    c = np.ascontiguousarray(coords, dtype=np.int64)
    v = np.ascontiguousarray(vals, dtype=np.float64)
    rank = int(np.asarray(factors[0]).shape[1])
    keep, arr = _factor_ptrs(factors, rank, d)
    out = np.zeros((int(d[mode]), rank), dtype=np.float64)
    used = _P().par_mttkrp(len(d), _ptr(d), v.shape[0], _ptr(c), _ptr(v), rank, arr, int(mode), _ptr(out))
    if used < 0:
        raise ValueError("invalid mode or rank, or out of memory")
    del keep
    return out, used


def _L():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build_oracle(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64 = ctypes.c_int64
        lib.oracle_plan.argtypes = [ctypes.c_int, P, P, P, P]
        lib.oracle_plan.restype = ctypes.c_int
        lib.oracle_encode.argtypes = [ctypes.c_int, P, i64, P, P]
        lib.oracle_encode.restype = i64
        lib.oracle_decode.argtypes = [ctypes.c_int, P, i64, P, P]
        lib.oracle_decode.restype = ctypes.c_int
        lib.oracle_order.argtypes = [i64, P, P]
        lib.oracle_order.restype = ctypes.c_int
        lib.oracle_partition.argtypes = [ctypes.c_int, P, i64, P, i64, P, P]
        lib.oracle_partition.restype = ctypes.c_int
        lib.oracle_mttkrp.argtypes = [ctypes.c_int, P, i64, P, P, ctypes.c_int, P, ctypes.c_int, P]
        lib.oracle_mttkrp.restype = ctypes.c_int
        lib.oracle_mttkrp_rows.argtypes = [ctypes.c_int, P, i64, P, P, ctypes.c_int, P, ctypes.c_int, i64, P, P]
        lib.oracle_mttkrp_rows.restype = ctypes.c_int
        lib.oracle_phi.argtypes = [ctypes.c_int, P, i64, P, P, ctypes.c_int, P, P, ctypes.c_int, ctypes.c_double, P]
        lib.oracle_phi.restype = ctypes.c_int
        lib.oracle_pi.argtypes = [ctypes.c_int, i64, P, ctypes.c_int, P, ctypes.c_int, P]
        lib.oracle_pi.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _dims(dims) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(dims, dtype=np.uint64))


def plan(dims):
    """(B, nbits[N], pos[N,64], masks[N] as Python ints) of the ALTO index."""
    d = _dims(dims)
    n = len(d)
    nbits = np.zeros(n, dtype=np.int32)
    pos = np.zeros((n, 64), dtype=np.int32)
    masks = np.zeros((n, 2), dtype=np.uint64)
    total = _L().oracle_plan(n, _ptr(d), _ptr(nbits), _ptr(pos), _ptr(masks))
    if total < 0:
        raise ValueError("invalid dimensions or index wider than 128 bits")
    m = [int(masks[k, 0]) | (int(masks[k, 1]) << 64) for k in range(n)]
    return total, nbits, pos, m


def encode(dims, coords: np.ndarray) -> np.ndarray:
    """ALTO index of every nonzero as an (M, 2) uint64 array (lo, hi)."""
    d = _dims(dims)
    c = np.ascontiguousarray(coords, dtype=np.int64)
    m = c.shape[1]
    keys = np.zeros((m, 2), dtype=np.uint64)
    rc = _L().oracle_encode(len(d), _ptr(d), m, _ptr(c), _ptr(keys))
    if rc != 0:
        raise ValueError(f"coordinate out of range at nonzero {rc - 1}" if rc > 0 else "invalid dimensions")
    return keys


def decode(dims, keys: np.ndarray) -> np.ndarray:
    d = _dims(dims)
    k = np.ascontiguousarray(keys, dtype=np.uint64)
    m = k.shape[0]
    out = np.zeros((len(d), m), dtype=np.int64)
    if _L().oracle_decode(len(d), _ptr(d), m, _ptr(k), _ptr(out)) != 0:
        raise ValueError("invalid dimensions")
    return out


def order(keys: np.ndarray) -> np.ndarray:
    """Stable ordering permutation of the nonzeros by ALTO index."""
    k = np.ascontiguousarray(keys, dtype=np.uint64)
    m = k.shape[0]
    perm = np.zeros(m, dtype=np.int64)
    if _L().oracle_order(m, _ptr(k), _ptr(perm)) != 0:
        raise MemoryError("oracle_order")
    return perm


def partition(dims, sorted_keys: np.ndarray, nseg: int):
    """(starts[L+1], intervals[L, N, 2]) of ``nseg`` balanced line segments."""
    d = _dims(dims)
    k = np.ascontiguousarray(sorted_keys, dtype=np.uint64)
    m = k.shape[0]
    starts = np.zeros(nseg + 1, dtype=np.int64)
    iv = np.zeros((nseg, len(d), 2), dtype=np.uint64)
    if _L().oracle_partition(len(d), _ptr(d), m, _ptr(k), int(nseg), _ptr(starts), _ptr(iv)) != 0:
        raise ValueError("invalid partition request")
    return starts, iv


def _factor_ptrs(factors, rank, dims):
    fs = []
    for n, f in enumerate(factors):
        f = np.ascontiguousarray(f, dtype=np.float64)
        if f.shape != (int(dims[n]), rank):
            raise ValueError(f"factor {n} has shape {f.shape}, expected {(int(dims[n]), rank)}")
        fs.append(f)
    arr = (ctypes.c_void_p * len(fs))(*[f.ctypes.data for f in fs])
    return fs, arr


def mttkrp(dims, coords: np.ndarray, vals: np.ndarray, factors, mode: int) -> np.ndarray:
    """FP64 MTTKRP of mode ``mode``: X_(mode) times the Khatri-Rao product of
    the other factors, as a plain loop over the COO nonzeros."""
    d = _dims(dims)
    c = np.ascontiguousarray(coords, dtype=np.int64)
    v = np.ascontiguousarray(vals, dtype=np.float64)
    rank = int(np.asarray(factors[0]).shape[1])
    keep, arr = _factor_ptrs(factors, rank, d)
    out = np.zeros((int(d[mode]), rank), dtype=np.float64)
    rc = _L().oracle_mttkrp(len(d), _ptr(d), v.shape[0], _ptr(c), _ptr(v), rank, arr, int(mode), _ptr(out))
    if rc != 0:
        raise ValueError("invalid mode or rank")
    del keep
    return out


def mttkrp_rows(dims, coords, vals, factors, mode: int, rows) -> np.ndarray:
    """Rows ``rows`` (sorted, distinct) of the FP64 MTTKRP of mode ``mode``."""
    d = _dims(dims)
    c = np.ascontiguousarray(coords, dtype=np.int64)
    v = np.ascontiguousarray(vals, dtype=np.float64)
    r = np.ascontiguousarray(rows, dtype=np.int64)
    if r.size > 1 and not np.all(np.diff(r) > 0):
        raise ValueError("rows must be sorted and distinct")
    rank = int(np.asarray(factors[0]).shape[1])
    keep, arr = _factor_ptrs(factors, rank, d)
    out = np.zeros((r.shape[0], rank), dtype=np.float64)
    rc = _L().oracle_mttkrp_rows(
        len(d), _ptr(d), v.shape[0], _ptr(c), _ptr(v), rank, arr, int(mode), r.shape[0], _ptr(r), _ptr(out)
    )
    if rc != 0:
        raise ValueError("invalid mode or rank")
    del keep
    return out


def mttkrp_abs(dims, coords, vals, factors, mode: int, rows=None) -> np.ndarray:
    """Entry scale of the MTTKRP sum: S[i, r] = sum over the nonzeros x of row
    i of |val(x) * prod_{m != mode} A^(m)[i_m(x), r]|, i.e. the MTTKRP of the
    absolute values.  A floating-point evaluation of the sum in any order with
    unit roundoff u and at most k roundings per term errs by at most about
    k*u*S per entry, so S is the per-entry yardstick for rounding error
    (Higham, "Accuracy and Stability of Numerical Algorithms", ch. 4).
    ``rows`` restricts it to sampled rows as ``mttkrp_rows`` does."""
    av = np.abs(np.asarray(vals, dtype=np.float64))
    af = [np.abs(np.asarray(f, dtype=np.float64)) for f in factors]
    if rows is None:
        return mttkrp(dims, coords, av, af, mode)
    return mttkrp_rows(dims, coords, av, af, mode, rows)


def phi(dims, coords, vals, factors, B, mode: int, eps: float) -> np.ndarray:
    """FP64 CP-APR model update Phi of mode ``mode`` (Algorithm
    "alg:cp-apr-mu", Phi line): for every nonzero, the Khatri-Rao row krp of
    the other factors, the model value d = B(i_mode, :) . krp, and
    Phi(i_mode, :) += v / max(d, eps) * krp.  A plain loop over the COO
    nonzeros (alto_oracle.c)."""
    d = _dims(dims)
    c = np.ascontiguousarray(coords, dtype=np.int64)
    v = np.ascontiguousarray(vals, dtype=np.float64)
    rank = int(np.asarray(B).shape[1])
    keep, arr = _factor_ptrs([f if m != mode else np.zeros((int(d[m]), rank)) for m, f in enumerate(factors)],
                             rank, d)
    b = np.ascontiguousarray(B, dtype=np.float64)
    if b.shape != (int(d[mode]), rank):
        raise ValueError("B must be dims[mode] x rank")
    out = np.zeros((int(d[mode]), rank), dtype=np.float64)
    rc = _L().oracle_phi(len(d), _ptr(d), v.shape[0], _ptr(c), _ptr(v), rank, arr, _ptr(b), int(mode), float(eps),
                         _ptr(out))
    if rc != 0:
        raise ValueError("invalid mode or rank")
    del keep
    return out


def pi_rows(dims, coords, factors, mode: int) -> np.ndarray:
    """Pi of mode ``mode`` restricted to the nonzeros (Algorithm
    "alg:cp-apr-mu", Pi line): row x = Hadamard product of the other
    factors' rows at nonzero x, in input order."""
    d = _dims(dims)
    c = np.ascontiguousarray(coords, dtype=np.int64)
    rank = int(np.asarray(factors[0 if mode else 1]).shape[1])
    keep, arr = _factor_ptrs([f if m != mode else np.zeros((int(d[m]), rank)) for m, f in enumerate(factors)],
                             rank, d)
    out = np.zeros((c.shape[1], rank), dtype=np.float64)
    if _L().oracle_pi(len(d), c.shape[1], _ptr(c), rank, arr, int(mode), _ptr(out)) != 0:
        raise ValueError("invalid mode or rank")
    del keep
    return out


def _solve_spd_or_pinv(V: np.ndarray, M: np.ndarray):
    """Return (M V^+, used_cholesky).  V^+ is applied through a Cholesky
    factorisation when V is symmetric positive definite with no pivot
    L_ii^2 at or below R*eps*max(diag V), else through the symmetric
    eigendecomposition with eigenvalues at or below R*eps*max|eig| dropped."""
    R = V.shape[0]
    eps = np.finfo(np.float64).eps
    try:
        L = np.linalg.cholesky(V)
        # a pivot at rounding level means V is singular in exact arithmetic
        if np.min(np.diag(L)) ** 2 <= R * eps * np.max(np.diag(V)):
            raise np.linalg.LinAlgError("numerically singular")
        # A V = M  <=>  V A^T = M^T  (V symmetric)
        Y = np.linalg.solve(L, M.T)
        X = np.linalg.solve(L.T, Y)
        return X.T, True
    except np.linalg.LinAlgError:
        w, Q = np.linalg.eigh(V)
        cut = R * eps * max(float(np.max(np.abs(w))), 0.0)
        inv = np.where(w > cut, 1.0 / np.where(w > cut, w, 1.0), 0.0)
        return (M @ Q) * inv @ Q.T, False


def als_sweep(dims, coords, vals, factors, return_mttkrp: bool = False):
    """One CP-ALS sweep (all modes, in order 0..N-1) in FP64.

    For each mode n: Grams of the other factors, V = their Hadamard product,
    M = MTTKRP(n), A^(n) = M V^+ (Cholesky, pseudo-inverse fallback),
    lambda = column 2-norms of A^(n), columns divided by lambda (a zero
    column stays zero with lambda = 0).  Returns (factors, lambda of the last
    mode, per-mode flags of whether Cholesky succeeded[, per-mode M])."""
    A = [np.array(f, dtype=np.float64, copy=True) for f in factors]
    N = len(A)
    R = A[0].shape[1]
    lam = np.zeros(R)
    chol_ok = []
    Ms = []
    for n in range(N):
        V = np.ones((R, R))
        for m in range(N):
            if m != n:
                V *= A[m].T @ A[m]
        M = mttkrp(dims, coords, vals, A, n)
        if return_mttkrp:
            Ms.append(M)
        An, ok = _solve_spd_or_pinv(V, M)
        chol_ok.append(ok)
        lam = np.sqrt(np.sum(An * An, axis=0))
        safe = np.where(lam > 0, lam, 1.0)
        A[n] = An / safe
    if return_mttkrp:
        return A, lam, chol_ok, Ms
    return A, lam, chol_ok


def tensor_norm2(dims, coords, vals) -> float:
    """||X||_F^2 of the tensor the nonzeros add up to: duplicate coordinates
    are summed first (a nonzero list with repeats stands for their sum)."""
    c = np.ascontiguousarray(np.asarray(coords, dtype=np.int64).T)
    v = np.asarray(vals, dtype=np.float64)
    if v.size == 0:
        return 0.0
    _, inv = np.unique(c, axis=0, return_inverse=True)
    s = np.bincount(inv.ravel(), weights=v)
    return float(np.dot(s, s))


def cp_fit(dims, coords, vals, factors, lam, xnorm2=None) -> float:
    """Fit 1 - ||X - Xhat||_F / ||X||_F of the CP model
    Xhat = sum_r lam_r a_r^(0) o ... o a_r^(N-1), the quantity whose
    improvement Algorithm "alg:cp-als" watches.  Expanded as
    ||X - Xhat||^2 = ||X||^2 + lam^T (Hadamard of the Grams A^(m)T A^(m)) lam
    - 2 sum_r lam_r <M(:, r), A^(N-1)(:, r)>, with M the MTTKRP of the last
    mode (the inner product of X with each rank-one term)."""
    A = [np.asarray(f, dtype=np.float64) for f in factors]
    lam = np.asarray(lam, dtype=np.float64)
    N = len(A)
    R = A[0].shape[1]
    xx = tensor_norm2(dims, coords, vals) if xnorm2 is None else float(xnorm2)
    G = np.ones((R, R))
    for m in range(N):
        G *= A[m].T @ A[m]
    hh = float(lam @ G @ lam)
    M = mttkrp(dims, coords, vals, A, N - 1)
    xh = float(np.sum(lam * np.sum(M * A[N - 1], axis=0)))
    r2 = max(xx + hh - 2.0 * xh, 0.0)
    return 1.0 - np.sqrt(r2) / np.sqrt(xx) if xx > 0 else 0.0


def cp_als(dims, coords, vals, factors, max_sweeps: int, tol: float):
    """Algorithm "alg:cp-als": CP-ALS sweeps until the fit changes by less
    than ``tol`` from one sweep to the next ("until fit ceases to improve"),
    at most ``max_sweeps``.  Returns (factors, lambda, fits per sweep)."""
    A = [np.array(f, dtype=np.float64, copy=True) for f in factors]
    xx = tensor_norm2(dims, coords, vals)
    fits = []
    lam = np.zeros(A[0].shape[1])
    for _ in range(max_sweeps):
        A, lam, _ = als_sweep(dims, coords, vals, A)
        fits.append(cp_fit(dims, coords, vals, A, lam, xnorm2=xx))
        if len(fits) > 1 and abs(fits[-1] - fits[-2]) < tol:
            break
    return A, lam, fits


def poisson_objective(dims, coords, vals, factors, lam) -> float:
    """Negative Poisson log-likelihood of the model [lam; A^(0..N-1)] for the
    count tensor the nonzeros add up to, up to the constant sum(log x!):
    sum over all entries of the model minus sum over the nonzeros of
    x log(model).  The model's total is sum_r lam_r prod_m (column sum of
    A^(m)(:, r)).  Duplicate coordinates are summed first."""
    c = np.ascontiguousarray(coords, dtype=np.int64)
    v = np.asarray(vals, dtype=np.float64)
    lam = np.asarray(lam, dtype=np.float64)
    total = float(np.sum(lam * np.prod([np.asarray(f, dtype=np.float64).sum(axis=0) for f in factors], axis=0)))
    if c.shape[1] == 0:
        return total
    flat = np.ravel_multi_index(tuple(c), tuple(int(d) for d in dims))
    cells, inv = np.unique(flat, return_inverse=True)
    x = np.bincount(inv, weights=v)
    first = np.zeros(len(cells), dtype=np.int64)
    first[inv[::-1]] = np.arange(c.shape[1])[::-1]
    model = np.ones((len(cells), lam.shape[0])) * lam[None, :]
    for m, f in enumerate(factors):
        model *= np.asarray(f, dtype=np.float64)[c[m, first]]
    mv = model.sum(axis=1)
    return total - float(np.sum(x * np.log(mv)))


def cp_apr_mu(dims, coords, vals, factors, lam=None, k_max: int = 10, l_max: int = 10, tau: float = 1e-4,
              kappa: float = 1e-2, kappa_tol: float = 1e-10, eps: float = 1e-10):
    """Algorithm "alg:cp-apr-mu" (CP-APR by multiplicative updates) in FP64,
    step by step: for each outer iteration k and mode n, S (the
    inadmissible-zero adjustment: kappa where k > 1, A^(n) < kappa_tol and the
    mode's last Phi exceeds 1), B = (A^(n) + S) Lambda, then up to l_max
    inner iterations of Phi (``phi``, the Pi rows formed on the fly), the KKT
    check max|min(B, 1 - Phi)| < tau, and B = B * Phi; finally lambda = the
    column sums of B and A^(n) = B Lambda^-1 (a zero column stays zero).  The
    outer loop stops early when no mode needed an update.  lam defaults to
    ones.  Returns (factors, lam, outer iterations run, inner iterations per
    outer iteration and mode, converged)."""
    A = [np.array(f, dtype=np.float64, copy=True) for f in factors]
    N = len(A)
    R = A[0].shape[1]
    lam = np.ones(R) if lam is None else np.array(lam, dtype=np.float64, copy=True)
    last_phi = [None] * N
    inner = []
    converged = False
    k = 0
    for k in range(1, k_max + 1):
        converged = True
        counts = []
        for n in range(N):
            S = np.zeros_like(A[n])
            if k > 1:
                S[(A[n] < kappa_tol) & (last_phi[n] > 1.0)] = kappa
            B = (A[n] + S) * lam[None, :]
            runs = 0
            for _ in range(l_max):
                last_phi[n] = phi(dims, coords, vals, A, B, n, eps)
                runs += 1
                if np.max(np.abs(np.minimum(B, 1.0 - last_phi[n]))) < tau:
                    break
                converged = False
                B = B * last_phi[n]
            lam = B.sum(axis=0)
            A[n] = B / np.where(lam > 0, lam, 1.0)[None, :]
            counts.append(runs)
        inner.append(counts)
        if converged:
            break
    return A, lam, k, inner, converged
