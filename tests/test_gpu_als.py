"""GPU CP-ALS sweep parity with the FP64 oracle."""

import numpy as np
import pytest

import oracle
from gpu_cases import bf16_round, case, factors_for, rel_fro, say, upload, vals32
from sweep_check import check_sweep
from test_oracle_mttkrp import exact_low_rank

pytestmark = pytest.mark.gpu

alto = pytest.importorskip("paper_2403_06348_amd")
torch = pytest.importorskip("torch")


def oracle_mode_update(X, cur, n, quantize=False):
    """One mode update of Algorithm "alg:cp-als" in FP64 from the factors the
    GPU held when it updated mode n (Grams from FP32 masters; MTTKRP from the
    BF16-rounded factors when ``quantize``)."""
    v = vals32(X).astype(np.float64)
    f64 = [c.astype(np.float64) for c in cur]
    fm = [bf16_round(c).astype(np.float64) for c in cur] if quantize else f64
    R = cur[0].shape[1]
    V = np.ones((R, R))
    for m in range(X.nmodes):
        if m != n:
            V *= f64[m].T @ f64[m]
    M = oracle.mttkrp(X.dims, X.coords, v, fm, n)
    An, ok = oracle._solve_spd_or_pinv(V, M)
    lam = np.linalg.norm(An, axis=0)
    return An / np.where(lam > 0, lam, 1.0), lam, ok, V, M


def lam_weighted_err(got, ref, lam):
    """Relative Frobenius error of got * diag(lam) against ref * diag(lam)."""
    return rel_fro(got.astype(np.float64) * lam, ref * lam)


@pytest.mark.parametrize("name,rank,fdt", [("c1", 8, "f32"), ("c2s", 16, "f32"), ("c3s", 32, "f32"),
                                           ("c2s", 64, "bf16"), ("w128", 16, "f32"), ("c1", 6, "f32"),
                                           ("c2s", 10, "f32"), ("c3s", 5, "bf16")])
def test_sweep_per_mode_parity(name, rank, fdt):
    """Every mode of one sweep against the oracle's update from the factors
    that mode saw (ranks 5, 6 and 10 run zero-padded to a multiple of 4)."""
    X = case(name)
    coords, vals = upload(X)
    T = alto.AltoTensor(X.dims, coords, vals)
    facs = factors_for(X, rank, seed=21)
    gf = [torch.from_numpy(f.copy()).cuda() for f in facs]
    say(f"[als] sweep {name} R={rank} {fdt}")
    lam = T.sweep(gf, fdt=alto.BF16 if fdt == "bf16" else alto.F32)
    torch.cuda.synchronize()
    assert T.sweep_flags() == 0
    assert lam.shape[0] == rank
    new = [g.cpu().numpy() for g in gf]
    check_sweep(X.dims, X.coords, vals32(X), facs, new, lam.cpu().numpy(), what=f"{name} R={rank}",
                quantize=(fdt == "bf16"))
    T.free()


def test_sweep_matches_whole_oracle_sweep_small():
    X = case("c1")
    coords, vals = upload(X)
    T = alto.AltoTensor(X.dims, coords, vals)
    facs = factors_for(X, 8, seed=3)
    gf = [torch.from_numpy(f.copy()).cuda() for f in facs]
    say("[als] whole sweep c1")
    lam = T.sweep(gf)
    A, lam_ref, ok = oracle.als_sweep(X.dims, X.coords, vals32(X).astype(np.float64),
                                      [f.astype(np.float64) for f in facs])
    for n in range(3):
        assert rel_fro(gf[n].cpu().numpy().astype(np.float64), A[n]) <= 1e-4
    assert rel_fro(lam.cpu().numpy(), lam_ref) <= 1e-4
    T.free()


def test_sweep_fixed_point_exact_rank():
    dims = (40, 50, 60)
    facs, lam_true, coords, vals = exact_low_rank(dims, 8, seed=4)
    T = alto.AltoTensor(dims, torch.from_numpy(coords).cuda(), torch.from_numpy(vals.astype(np.float32)).cuda())
    gf = [torch.from_numpy(f.astype(np.float32)).cuda() for f in facs]
    say("[als] fixed point")
    lam = T.sweep(gf)
    for n in range(3):
        assert rel_fro(gf[n].cpu().numpy().astype(np.float64), facs[n]) <= 1e-5
    assert rel_fro(lam.cpu().numpy(), lam_true) <= 1e-5
    T.free()


@pytest.mark.parametrize("name,rank", [("c1", 8), ("c2s", 32), ("c2s", 64)])
def test_sweep_pseudoinverse_fallback(name, rank):
    X = case(name)
    coords, vals = upload(X)
    T = alto.AltoTensor(X.dims, coords, vals)
    facs = factors_for(X, rank, seed=5)
    for n in (1, 2):
        facs[n][:, 3] = facs[n][:, 2]
    gf = [torch.from_numpy(f.copy()).cuda() for f in facs]
    say(f"[als] pseudo-inverse fallback {name} R={rank}")
    T.sweep(gf)
    flags = T.sweep_flags()
    assert flags & 1
    got0 = gf[0].cpu().numpy().astype(np.float64)
    ref0, _, ok, _, _ = oracle_mode_update(X, facs, 0)
    assert not ok
    assert rel_fro(got0, ref0) <= 1e-4
    T.free()


def test_sweep_graph_capture_replays_match_eager():
    """The whole sweep captured in one HIP graph; every replay is checked
    against an eager sweep from the same factors, with eager work and
    synchronizations between the replays."""
    X = case("c2s")
    coords, vals = upload(X)
    T = alto.AltoTensor(X.dims, coords, vals)
    facs = factors_for(X, 16, seed=8)
    gf = [torch.from_numpy(f.copy()).cuda() for f in facs]
    lam = torch.empty(16, dtype=torch.float64, device="cuda")
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        T.sweep([g.clone() for g in gf], lam=lam)  # allocates the workspace
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    start = [g.clone() for g in gf]
    say("[als] capture sweep")
    with torch.cuda.graph(graph, stream=side):
        T.sweep(gf, lam=lam)
    torch.cuda.synchronize()
    for g, s0 in zip(gf, start):
        g.copy_(s0)
    eager = [g.clone() for g in start]
    eager_lam = torch.empty_like(lam)
    for rep in range(3):
        before = [g.cpu().numpy().astype(np.float64) for g in gf]
        graph.replay()
        torch.cuda.synchronize()
        T.sweep(eager, lam=eager_lam)  # eager sweep from the same state
        torch.cuda.synchronize()
        after = [g.cpu().numpy().astype(np.float64) for g in gf]
        for n in range(X.nmodes):
            # V of mode n from the factors both runs held at that point
            cur = [after[m] if m < n else before[m] for m in range(X.nmodes)]
            _, ref_lam, _, V, _ = oracle_mode_update(X, [c.astype(np.float32) for c in cur], n)
            # both unnormalized updates are within the MTTKRP gate (1e-5) of
            # the exact one, amplified by cond(V); they differ only in FP32
            # summation order (columns weighted by lambda, as above)
            tol = max(1e-5, 2e-5 * np.linalg.cond(V))
            e = lam_weighted_err(after[n], eager[n].cpu().numpy().astype(np.float64), ref_lam)
            say(f"    replay {rep} mode {n}: rel diff {e:.2e} (tol {tol:.1e})")
            assert e <= tol
        assert rel_fro(lam.cpu().numpy(), eager_lam.cpu().numpy()) <= tol
        for g, ge in zip(gf, eager):  # continue both from the same state
            ge.copy_(g)
    T.free()
