"""CP-APR by multiplicative updates on the GPU (alto_cpapr_mu) against the
oracle's Algorithm "alg:cp-apr-mu": the same outer/inner iteration counts,
factors and lambda on a c3-style count tensor (Poisson(3)+1 values, Zipf and
uniform modes), the exact fixed point of a disjoint-support model, and the
argument checks."""

import numpy as np
import pytest

import oracle
from gpu_cases import rel_fro, say, vals32
from synth import make_factors, zipf_tensor

pytestmark = pytest.mark.gpu

alto = pytest.importorskip("paper_2403_06348_amd")
torch = pytest.importorskip("torch")


def _upload(X):
    return alto.AltoTensor(X.dims, torch.from_numpy(X.coords).cuda(), torch.from_numpy(vals32(X)).cuda())


@pytest.mark.parametrize("R,pi_form", [(8, 1), (8, 2), (16, 0)])
def test_cpapr_matches_oracle_iterations_and_factors(R, pi_form):
    """pi_form 1: Pi precomputed (ALTO-PRE), 2: on the fly (ALTO-OTF), 0: the
    library's rule (PRE for this 4-mode tensor at l_max = 10)."""
    X = zipf_tensor((50_000, 512, 256, 3_000), 300_000, (1.1, None, None, 1.1), seed=13 + R,
                    vals="poisson3p1_f32", name="apr")
    T = _upload(X)
    start = [0.1 + f for f in make_factors(X.dims, R, seed=R)]  # strictly positive
    fa = [torch.from_numpy(np.ascontiguousarray(f, dtype=np.float32)).cuda() for f in start]
    lam = torch.ones(R, dtype=torch.float64, device="cuda")
    prm = dict(k_max=2, l_max=10, tau=1e-4, kappa=1e-2, kappa_tol=1e-10, eps=1e-10)
    say(f"[cpapr] R={R} pi_form={pi_form}: GPU")
    k, counts, conv = T.cpapr_mu(fa, lam, pi_form=pi_form, **prm)
    say(f"[cpapr] R={R}: oracle")
    A, lam_o, k_o, counts_o, conv_o = oracle.cp_apr_mu(X.dims, X.coords, vals32(X).astype(np.float64),
                                                       [f.astype(np.float32).astype(np.float64) for f in start],
                                                       **prm)
    say(f"    outer {k} / {k_o}, inner {counts} / {counts_o}")
    assert (k, counts, conv) == (k_o, counts_o, conv_o)
    # every Phi evaluation carries FP32 rounding of B, Phi and the factors
    # (about 1e-7 relative each); the multiplicative updates add these up
    # over the k_max * N * l_max evaluations: 2 * 4 * 10 * 1e-7 = 8e-6, so
    # 1e-5 relative Frobenius per factor, and for lambda (measured: 1e-7)
    for n in range(X.nmodes):
        e = rel_fro(fa[n].cpu().numpy().astype(np.float64), A[n])
        say(f"    mode {n}: factor rel err {e:.2e}")
        assert e <= 1e-5
    el = rel_fro(lam.cpu().numpy(), lam_o)
    say(f"    lambda rel err {el:.2e}")
    assert el <= 1e-5
    T.free()


def test_cpapr_fixed_point_of_an_exact_model():
    """Rank 4 with disjoint column supports, each column summing to 1, and
    the tensor equal to the model on the support: Phi = 1 there, every mode
    converges at its first inner iteration, nothing changes."""
    rng = np.random.default_rng(2)
    blocks = [((0, 2), (0, 3), (0, 2)), ((2, 5), (3, 5), (2, 3)), ((5, 6), (5, 8), (3, 6)), ((6, 9), (8, 9), (6, 8))]
    dims = (9, 9, 8)
    R = 4
    facs = [np.zeros((d, R)) for d in dims]
    for r, blk in enumerate(blocks):
        for m, (a, b) in enumerate(blk):
            w = rng.uniform(0.5, 1.5, b - a)
            facs[m][a:b, r] = w / w.sum()
    lam0 = np.array([20.0, 7.0, 13.0, 5.0])
    cells, vals = [], []
    for r, blk in enumerate(blocks):
        for i in range(*blk[0]):
            for j in range(*blk[1]):
                for k in range(*blk[2]):
                    cells.append((i, j, k))
                    vals.append(lam0[r] * facs[0][i, r] * facs[1][j, r] * facs[2][k, r])
    coords = np.ascontiguousarray(np.array(cells, dtype=np.int64).T)
    v32 = np.array(vals, dtype=np.float32)
    f32 = [f.astype(np.float32) for f in facs]
    T = alto.AltoTensor(dims, torch.from_numpy(coords).cuda(), torch.from_numpy(v32).cuda())
    fa = [torch.from_numpy(f.copy()).cuda() for f in f32]
    lam = torch.from_numpy(lam0.copy()).cuda()
    k, counts, conv = T.cpapr_mu(fa, lam, k_max=5, l_max=10, tau=1e-5)
    assert conv and k == 1 and counts == [[1, 1, 1]]
    for n in range(3):
        np.testing.assert_allclose(fa[n].cpu().numpy(), f32[n], rtol=0, atol=1e-6)
    np.testing.assert_allclose(lam.cpu().numpy(), lam0, rtol=1e-5)
    T.free()


def test_cpapr_argument_errors():
    X = zipf_tensor((300, 200, 100), 5_000, (1.2, None, None), seed=3, vals="poisson3p1_f32", name="aprerr")
    T = _upload(X)
    f6 = [torch.rand((d, 6), device="cuda") for d in X.dims]
    with pytest.raises(alto.AltoError):
        T.cpapr_mu(f6, torch.ones(6, dtype=torch.float64, device="cuda"))
    f8 = [torch.rand((d, 8), device="cuda") for d in X.dims]
    with pytest.raises(alto.AltoError):
        T.cpapr_mu(f8, torch.ones(8, dtype=torch.float64, device="cuda"), k_max=0)
    with pytest.raises(alto.AltoError):
        T.cpapr_mu(f8, torch.ones(8, dtype=torch.float64, device="cuda"), eps=0.0)
    T.free()
