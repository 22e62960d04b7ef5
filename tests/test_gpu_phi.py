"""CP-APR model update Phi (Algorithm "alg:cp-apr-mu", Phi line; Algorithm
"fig:subproblem_algo") on the GPU against the FP64 oracle, entry by entry,
with Pi formed on the fly (ALTO-OTF) and precomputed (ALTO-PRE).  Inputs are
positive (values, factors and B), so every term of an entry is positive and
the entry itself is the scale of its rounding error."""

import numpy as np
import pytest

import oracle
from gpu_cases import assert_entrywise, case, factors_for, rel_fro, say, upload, vals32

pytestmark = pytest.mark.gpu

alto = pytest.importorskip("paper_2403_06348_amd")
torch = pytest.importorskip("torch")

_built = {}


def built(name):
    if name not in _built:
        X = case(name)
        coords, vals = upload(X)
        _built[name] = (X, alto.AltoTensor(X.dims, coords, vals))
    return _built[name]


def b_for(X, n, R, seed=0):
    return np.random.default_rng(100 + seed + n).uniform(0.1, 1.0, (X.dims[n], R)).astype(np.float32)


PLANS = {
    "default": None,
    "tile_small": dict(conflict=alto.CR_TILE, tile_nnz=1000, table_slots=64),
    "run": dict(conflict=alto.CR_RUN),
    "f64": dict(accumulate=alto.ACC_F64),
}


@pytest.mark.parametrize("name,rank", [("c1", 8), ("c2s", 16), ("c3s", 32), ("w128", 8), ("unit", 12)])
@pytest.mark.parametrize("plan", list(PLANS))
@pytest.mark.parametrize("pre", [False, True])
def test_phi_parity(name, rank, plan, pre):
    X, T = built(name)
    facs = factors_for(X, rank, seed=50)
    gf = [torch.from_numpy(f).cuda() for f in facs]
    v64 = vals32(X).astype(np.float64)
    f64 = [f.astype(np.float64) for f in facs]
    for n in range(X.nmodes):
        B = b_for(X, n, rank)
        pi = T.cpapr_pi(n, gf) if pre else None
        say(f"[phi] {name} R={rank} plan={plan} {'PRE' if pre else 'OTF'} mode {n}")
        got = T.cpapr_phi(n, gf, torch.from_numpy(B).cuda(), eps=1e-10, pi=pi,
                          plan=PLANS[plan]).cpu().numpy().astype(np.float64)
        ref = oracle.phi(X.dims, X.coords, v64, f64, B.astype(np.float64), n, 1e-10)
        w = assert_entrywise(got, ref, ref, what=f"phi {name} mode {n}")
        e = rel_fro(got, ref)
        say(f"    rel err {e:.2e}, worst entry {w:.2f} x tol")
        assert e <= 1e-5


@pytest.mark.parametrize("name,rank", [("c3s", 16), ("w128", 8)])
def test_pi_rows_in_alto_order(name, rank):
    X, T = built(name)
    facs = factors_for(X, rank, seed=51)
    gf = [torch.from_numpy(f).cuda() for f in facs]
    keys = oracle.encode(X.dims, X.coords)
    perm = np.lexsort((np.arange(X.nnz), keys[:, 0], keys[:, 1]))  # stable ALTO order
    for n in range(X.nmodes):
        got = T.cpapr_pi(n, gf).cpu().numpy().astype(np.float64)
        ref = oracle.pi_rows(X.dims, X.coords, [f.astype(np.float64) for f in facs], n)[perm]
        # N - 1 FP32 products per entry
        np.testing.assert_allclose(got, ref, rtol=X.nmodes * 2.0**-24, atol=0)


def test_phi_eps_floor():
    """B = 0: every denominator is eps, Phi = MTTKRP / eps."""
    X, T = built("c3s")
    R, eps = 8, 1e-3
    facs = factors_for(X, R, seed=52)
    gf = [torch.from_numpy(f).cuda() for f in facs]
    v64 = vals32(X).astype(np.float64)
    for n in range(X.nmodes):
        B = torch.zeros((X.dims[n], R), device="cuda")
        got = T.cpapr_phi(n, gf, B, eps=eps).cpu().numpy().astype(np.float64)
        ref = oracle.mttkrp(X.dims, X.coords, v64, [f.astype(np.float64) for f in facs], n) / eps
        assert_entrywise(got, ref, ref, what=f"eps floor mode {n}")


def test_phi_argument_errors():
    X, T = built("c1")
    gf = [torch.rand(d, 8, device="cuda") for d in X.dims]
    B = torch.rand(X.dims[0], 8, device="cuda")
    with pytest.raises(alto.AltoError):
        T.cpapr_phi(0, gf, B, eps=0.0)
    with pytest.raises(alto.AltoError):
        T.cpapr_phi(0, gf, torch.rand(X.dims[0], 6, device="cuda"))
    with pytest.raises(alto.AltoError):
        T.cpapr_phi(0, None, B)  # OTF needs the factors


def test_pre_otf_choice():
    """ALTO-PRE is chosen for low fiber reuse with factors far beyond the
    GPU's L2; ALTO-OTF otherwise (Sec. "Adaptive Memory Management")."""
    X, T = built("lowreuse")  # 3e6 x 2e6 x 4e6, 4e5 nonzeros: reuse < 1
    assert T.cpapr_prefer_pre(0, 16)
    X2, T2 = built("c2s")  # reuse 1.2 .. 12 with factors of 1e5 .. 1e6 rows
    assert not T2.cpapr_prefer_pre(2, 16)  # reuse 12
    X3, T3 = built("c1")
    assert not any(T3.cpapr_prefer_pre(n, 8) for n in range(3))  # factors fit in L2
