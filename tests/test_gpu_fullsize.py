"""Parity at the full workload sizes, in the launch configuration the bench
times (autotuned plans): the ordered ALTO tensor bit for bit, and MTTKRP on
sampled output rows (the heaviest rows and random ones), which the oracle
computes one by one in a single pass over the nonzeros."""

import numpy as np
import pytest

import oracle
from gpu_cases import ENTRY_TOL, assert_entrywise, bf16_round, rel_fro, say, vals32
from synth import CONFIGS, make_config, make_factors

pytestmark = pytest.mark.gpu

alto = pytest.importorskip("paper_2403_06348_amd")
torch = pytest.importorskip("torch")

_cache = {}


def full(name):
    if name not in _cache:
        say(f"[full] generating {name}")
        X = make_config(name)
        coords = torch.from_numpy(X.coords).cuda()
        vals = torch.from_numpy(vals32(X)).cuda()
        T = alto.AltoTensor(X.dims, coords, vals)
        del coords, vals
        _cache[name] = (X, T)
    return _cache[name]


def sample_rows(coords_n, dim, k_heavy=16, k_rand=200, seed=0):
    counts = np.bincount(coords_n, minlength=dim)
    heavy = np.argsort(counts)[::-1][:k_heavy]
    rnd = np.random.default_rng(seed).choice(dim, size=min(k_rand, dim), replace=False)
    return np.unique(np.concatenate([heavy, rnd]))


def test_full_c2_ordered_tensor_bitexact():
    X, T = full("c2")
    say("[full] c2 keys and values")
    keys, vals = T.export()
    torch.cuda.synchronize()
    ok = oracle.encode(X.dims, X.coords)[:, 0]
    perm = np.argsort(ok, kind="stable")
    np.testing.assert_array_equal(keys.cpu().numpy().view(np.uint64)[:, 0], ok[perm])
    np.testing.assert_array_equal(vals.cpu().numpy(), vals32(X)[perm])


@pytest.mark.parametrize("name", ["c2", "c3"])
def test_full_mttkrp_sampled_rows(name):
    X, T = full(name)
    R = CONFIGS[name]["rank"]
    facs = make_factors(X.dims, R, seed=7)
    gf = [torch.from_numpy(f).cuda() for f in facs]
    v64 = vals32(X).astype(np.float64)
    f64 = [f.astype(np.float64) for f in facs]
    for n in range(X.nmodes):
        out = torch.empty((X.dims[n], R), device="cuda")
        plan = T.autotune(n, gf, out=out)
        say(f"[full] {name} mode {n} plan {plan}")
        got = T.mttkrp(n, gf, out=out).cpu().numpy().astype(np.float64)
        rows = sample_rows(X.coords[n], X.dims[n], seed=n)
        ref = oracle.mttkrp_rows(X.dims, X.coords, v64, f64, n, rows)
        S = oracle.mttkrp_abs(X.dims, X.coords, v64, f64, n, rows=rows)
        e = rel_fro(got[rows], ref)
        w = assert_entrywise(got[rows], ref, S, what=f"{name} mode {n}")
        say(f"    {len(rows)} rows: rel err {e:.2e}, worst entry {w:.2f} x tol")
        assert e <= 1e-5


def test_full_c4_bf16_factors_sampled_rows():
    """Precision form at full size: the c2 tensor with R=64 factors stored as
    BF16, autotuned plans (rank tiles).  The oracle runs on the same
    BF16-rounded factors, so the bound is the FP32 accumulation's."""
    X, T = full("c2")  # the precision form's tensor is the c2 tensor
    R = CONFIGS["c4"]["rank"]
    facs = make_factors(X.dims, R, seed=7)
    gf = [torch.from_numpy(f).cuda().to(torch.bfloat16).view(torch.int16) for f in facs]
    v64 = vals32(X).astype(np.float64)
    f64 = [bf16_round(f).astype(np.float64) for f in facs]
    for n in range(X.nmodes):
        out = torch.empty((X.dims[n], R), device="cuda")
        plan = T.autotune(n, gf, out=out, rank=R, fdt=alto.BF16)
        say(f"[full] c4 mode {n} plan {plan}")
        got = T.mttkrp(n, gf, out=out, rank=R, fdt=alto.BF16).cpu().numpy().astype(np.float64)
        rows = sample_rows(X.coords[n], X.dims[n], seed=10 + n)
        ref = oracle.mttkrp_rows(X.dims, X.coords, v64, f64, n, rows)
        S = oracle.mttkrp_abs(X.dims, X.coords, v64, f64, n, rows=rows)
        e = rel_fro(got[rows], ref)
        w = assert_entrywise(got[rows], ref, S, what=f"c4 mode {n}")
        say(f"    {len(rows)} rows: rel err {e:.2e}, worst entry {w:.2f} x tol")
        assert e <= 1e-5


def _row_subsets(X, seed):
    """Per mode: sampled output rows (8 heavy rows below the very heaviest,
    64 random ones) and the nonzeros that land in them, so that each oracle
    call walks only those nonzeros (the other nonzeros add nothing to the
    sampled rows)."""
    subs = []
    for n in range(X.nmodes):
        counts = np.bincount(X.coords[n], minlength=X.dims[n])
        order = np.argsort(counts)[::-1]
        g = np.random.default_rng(seed + n)
        heavy = g.choice(order[8:200], size=8, replace=False)
        rnd = g.choice(X.dims[n], size=64, replace=False)
        rows = np.unique(np.concatenate([heavy, rnd]))
        keep = np.isin(X.coords[n], rows)
        subs.append((rows, np.ascontiguousarray(X.coords[:, keep]), vals32(X)[keep].astype(np.float64)))
    return subs


def test_full_c4_ten_sweeps_per_mttkrp_error():
    """The precision form over a whole run: 10 CP-ALS sweeps of the c2 tensor
    at R=64 with BF16 factor shadows.  Every MTTKRP of every sweep is redone
    from the exact inputs the sweep gave it (modes before n already updated,
    the others from the previous sweep, BF16-rounded) and checked on sampled
    rows against the oracle on the same BF16-rounded factors (Frobenius and
    per entry, 1e-5), and against the FP32-factor path, whose distance from
    it is bounded by the BF16 rounding of two factors per term."""
    X, T = full("c2")
    R = CONFIGS["c4"]["rank"]
    subs = _row_subsets(X, seed=40)
    work = [torch.from_numpy(f).cuda() for f in make_factors(X.dims, R, seed=7)]
    lam = torch.empty(R, dtype=torch.float64, device="cuda")
    u = 2.0**-8  # BF16 unit roundoff (8-bit significand)
    quant = ((1 + u) ** 2 - 1) / (1 - u) ** 2 + 2 * ENTRY_TOL
    for k in range(10):
        snap = [w.clone() for w in work]
        T.sweep(work, lam=lam, fdt=alto.BF16)
        errs, qerrs = [], []
        for n in range(X.nmodes):
            ins = [work[m] if m < n else snap[m] for m in range(X.nmodes)]
            bf = [f.to(torch.bfloat16) for f in ins]
            out = torch.empty((X.dims[n], R), device="cuda")
            got = T.mttkrp(n, [b.view(torch.int16) for b in bf], out=out, rank=R, fdt=alto.BF16)
            got = got.cpu().numpy().astype(np.float64)
            ref32 = T.mttkrp(n, ins, out=torch.empty_like(out)).cpu().numpy().astype(np.float64)
            rows, sc, sv = subs[n]
            f64 = [b.float().cpu().numpy().astype(np.float64) for b in bf]
            ref = oracle.mttkrp_rows(X.dims, sc, sv, f64, n, rows)
            S = oracle.mttkrp_abs(X.dims, sc, sv, f64, n, rows=rows)
            e = rel_fro(got[rows], ref)
            assert_entrywise(got[rows], ref, S, what=f"c4 sweep {k} mode {n}")
            assert e <= 1e-5, (k, n, e)
            # BF16 storage against the FP32-factor path: each term moves by at
            # most the rounding of its two factors
            assert_entrywise(got[rows], ref32[rows], S, tol=quant, what=f"c4 sweep {k} mode {n} vs FP32 path")
            errs.append(e)
            qerrs.append(rel_fro(got, ref32))
        say(f"[full] c4 sweep {k}: vs FP64 oracle {['%.2e' % e for e in errs]}, "
            f"vs FP32-factor path {['%.2e' % e for e in qerrs]}")
