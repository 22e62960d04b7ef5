"""GPU MTTKRP parity with the FP64 oracle: relative Frobenius error per mode
<= 1e-5 for FP32 factors, and every entry within 1e-5 of its own scale (the
sum of the absolute values of its terms); BF16 factors are compared with the
oracle run on the same BF16-rounded factors (accumulation error only)."""

import numpy as np
import pytest

import oracle
from gpu_cases import assert_entrywise, bf16_round, case, factors_for, rel_fro, say, upload, vals32

pytestmark = pytest.mark.gpu

alto = pytest.importorskip("paper_2403_06348_amd")
torch = pytest.importorskip("torch")

TOL = 1e-5

_built = {}


def built(name):
    if name not in _built:
        X = case(name)
        coords, vals = upload(X)
        _built[name] = (X, alto.AltoTensor(X.dims, coords, vals))
    return _built[name]


def oracle_modes(X, facs):
    v = vals32(X).astype(np.float64)
    f64 = [f.astype(np.float64) for f in facs]
    return [oracle.mttkrp(X.dims, X.coords, v, f64, n) for n in range(X.nmodes)]


_scales = []


def scale_of(X, facs, n):
    """Per-entry error scale of mode n; the last few are kept (with the
    factors they belong to, so that the identity check stays valid)."""
    for fx, fn, fm, S in _scales:
        if fx is X and fn is facs and fm == n:
            return S
    v = vals32(X).astype(np.float64)
    S = oracle.mttkrp_abs(X.dims, X.coords, v, [f.astype(np.float64) for f in facs], n)
    _scales.append((X, facs, n, S))
    del _scales[:-4]
    return S


def check(got, ref, X, facs, n, what):
    """Whole-result Frobenius bound and the per-entry bound."""
    err = rel_fro(got, ref)
    worst = assert_entrywise(got, ref, scale_of(X, facs, n), what=what)
    say(f"    rel err {err:.3e}  worst entry {worst:.2f} x tol")
    assert err <= TOL, (what, err)


PLANS = {
    "default": None,
    "tile_f32": dict(conflict=alto.CR_TILE, accumulate=alto.ACC_F32),
    "tile_f64_small": dict(conflict=alto.CR_TILE, accumulate=alto.ACC_F64, tile_nnz=1000, table_slots=64),
    "run_f64": dict(conflict=alto.CR_RUN, accumulate=alto.ACC_F64),
    "run_f32": dict(conflict=alto.CR_RUN, accumulate=alto.ACC_F32, tile_nnz=777),
    "hot": dict(conflict=alto.CR_HOT, accumulate=alto.ACC_F32),
    "hot_small": dict(conflict=alto.CR_HOT, accumulate=alto.ACC_F64, tile_nnz=1000, table_slots=64,
                      block_threads=256),
}


@pytest.mark.parametrize("name,rank", [("c1", 8), ("c2s", 16), ("c3s", 32), ("w128", 12), ("unit", 20),
                                       ("lowreuse", 16)])
@pytest.mark.parametrize("plan", list(PLANS))
def test_mttkrp_parity(name, rank, plan):
    X, T = built(name)
    facs = factors_for(X, rank)
    refs = oracle_modes(X, facs)
    gf = [torch.from_numpy(f).cuda() for f in facs]
    for n in range(X.nmodes):
        say(f"[mttkrp] {name} R={rank} plan={plan} mode={n}")
        got = T.mttkrp(n, gf, plan=PLANS[plan]).cpu().numpy().astype(np.float64)
        check(got, refs[n], X, facs, n, f"{name} R={rank} {plan} mode {n}")


@pytest.mark.parametrize("rank", [1, 3, 4, 6, 8, 10, 16, 24, 32, 33, 64, 128])
def test_mttkrp_ranks(rank):
    """Every rank from 1 to 128; ranks that are not a multiple of 4 run on
    zero-padded copies of the factors and output."""
    X, T = built("c2s")
    facs = factors_for(X, rank, seed=rank)
    refs = oracle_modes(X, facs)
    gf = [torch.from_numpy(f).cuda() for f in facs]
    for n in range(X.nmodes):
        say(f"[mttkrp] ranks R={rank} mode={n}")
        got = T.mttkrp(n, gf).cpu().numpy().astype(np.float64)
        check(got, refs[n], X, facs, n, f"c2s R={rank} mode {n}")


@pytest.mark.parametrize("name,rank", [("c2s", 16), ("c3s", 32), ("c2s", 64)])
def test_mttkrp_bf16_factors(name, rank):
    X, T = built(name)
    facs = factors_for(X, rank)
    rounded = [bf16_round(f) for f in facs]
    refs_q = oracle_modes(X, rounded)
    refs = oracle_modes(X, facs)
    bf = [torch.from_numpy(f).cuda().to(torch.bfloat16).view(torch.int16) for f in facs]
    for n in range(X.nmodes):
        say(f"[mttkrp] bf16 {name} R={rank} mode={n}")
        got = T.mttkrp(n, bf, rank=rank, fdt=alto.BF16).cpu().numpy().astype(np.float64)
        e_q = rel_fro(got, refs[n])
        check(got, refs_q[n], X, rounded, n, f"bf16 {name} R={rank} mode {n}")
        say(f"    vs oracle(fp32 factors) {e_q:.3e}")
        # quantisation: each factor entry carries at most 2^-9 relative error
        assert e_q <= (X.nmodes - 1) * 2.0**-8


def test_mttkrp_argument_errors():
    X, T = built("c1")
    gf = [torch.rand(d, 8, device="cuda") for d in X.dims]
    with pytest.raises(alto.AltoError):
        T.mttkrp(3, gf)
    with pytest.raises(alto.AltoError):
        T.mttkrp(0, gf, rank=0)
    with pytest.raises(alto.AltoError):
        T.mttkrp(0, gf, rank=129)
    with pytest.raises(alto.AltoError):
        T.mttkrp(0, [gf[0], None, gf[2]])
    with pytest.raises(alto.AltoError):
        T.mttkrp(0, gf, plan=dict(table_slots=100, conflict=alto.CR_TILE))
    with pytest.raises(alto.AltoError):
        T.mttkrp(0, gf, plan=dict(tile_order=3))


def test_autotune_records_a_plan_and_stays_exact():
    X, T = built("c2s")
    facs = factors_for(X, 16, seed=3)
    refs = oracle_modes(X, facs)
    gf = [torch.from_numpy(f).cuda() for f in facs]
    for n in range(X.nmodes):
        say(f"[mttkrp] autotune mode={n}")
        out = torch.empty((X.dims[n], 16), device="cuda")
        chosen = T.autotune(n, gf, out=out)
        assert chosen == T.get_plan(n, 16)
        check(out.cpu().numpy().astype(np.float64), refs[n], X, facs, n, f"autotune scratch mode {n}")
        got = T.mttkrp(n, gf).cpu().numpy().astype(np.float64)
        check(got, refs[n], X, facs, n, f"autotuned mode {n}")
    # a second handle of the same class starts from the cached plan
    coords, vals = upload(X)
    T2 = alto.AltoTensor(X.dims, coords, vals)
    assert T2.get_plan(2, 16) == T.get_plan(2, 16)
    T2.free()


def test_cached_plan_that_does_not_fit_falls_back():
    """The process-wide tuned-plan cache is keyed by a tensor class, within
    which a mode's length can differ by 4x.  A whole-mode-in-LDS plan tuned
    on a 520-row mode must not be used for a 2047-row mode of the same class
    (it would not fit the LDS): a plain call with no plan falls back to the
    default plan and stays exact."""
    from synth import zipf_tensor

    R = 32
    # same class: 3 modes, one index word, R=32, floor(log2 nnz) = 20 and
    # floor(log2 reuse of mode 2) = 10; mode 2 of B is 3.9x longer than A's
    A = zipf_tensor((3000, 2500, 520), 1 << 20, (1.2, 1.2, None), seed=41, name="classA")
    B = zipf_tensor((3000, 2500, 2047), (1 << 21) - 1, (1.2, 1.2, None), seed=42, name="classB")
    TA = alto.AltoTensor(A.dims, *upload(A))
    fa = [torch.from_numpy(f).cuda() for f in factors_for(A, R, seed=5)]
    chosen = TA.autotune(2, fa, out=torch.empty((A.dims[2], R), device="cuda"))
    say(f"[mttkrp] class A mode 2 tuned plan {chosen}")
    TB = alto.AltoTensor(B.dims, *upload(B))
    facs = factors_for(B, R, seed=6)
    fb = [torch.from_numpy(f).cuda() for f in facs]
    got = TB.mttkrp(2, fb).cpu().numpy().astype(np.float64)  # no plan: cache, else default
    pb = TB.get_plan(2, R)
    say(f"[mttkrp] class B mode 2 plan {pb}")
    if chosen["conflict"] == alto.CR_DIRECT:
        assert pb["conflict"] != alto.CR_DIRECT or pb["rank_tile"] not in (0, R)
    v64 = vals32(B).astype(np.float64)
    f64 = [f.astype(np.float64) for f in facs]
    ref = oracle.mttkrp(B.dims, B.coords, v64, f64, 2)
    S = oracle.mttkrp_abs(B.dims, B.coords, v64, f64, 2)
    assert rel_fro(got, ref) <= 1e-5
    assert_entrywise(got, ref, S, what="class B mode 2")
    TA.free()
    TB.free()


def test_mttkrp_graph_capture_replays_match_eager():
    """MTTKRP of every mode captured in one HIP graph; each replay, with eager
    work between replays, matches the eager result."""
    X, T = built("c2s")
    facs = [torch.from_numpy(f).cuda() for f in factors_for(X, 16, seed=12)]
    outs = [torch.empty((d, 16), device="cuda") for d in X.dims]
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        for n in range(X.nmodes):
            T.mttkrp(n, facs, out=outs[n])
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side):
        for n in range(X.nmodes):
            T.mttkrp(n, facs, out=outs[n])
    torch.cuda.synchronize()
    for rep in range(3):
        for o in outs:
            o.fill_(-1.0)
        graph.replay()
        torch.cuda.synchronize()
        for n in range(X.nmodes):
            eager = T.mttkrp(n, facs).cpu().numpy().astype(np.float64)
            e = rel_fro(outs[n].cpu().numpy().astype(np.float64), eager)
            say(f"[mttkrp] graph replay {rep} mode {n}: {e:.2e}")
            assert e <= 2e-5


@pytest.mark.parametrize("name,rank,mode,plan", [
    ("c3s", 32, 1, dict(conflict=alto.CR_DIRECT, rank_tile=8, block_threads=256)),
    # 2048 rows x 17 FP32 columns: 136 KiB of the 160 KiB LDS
    ("c3s", 32, 1, dict(conflict=alto.CR_DIRECT, rank_tile=16, block_threads=512)),
    # 1024 rows, all 32 columns in one pass
    ("c3s", 32, 2, dict(conflict=alto.CR_DIRECT, rank_tile=32, block_threads=512)),
    ("c3s", 32, 2, dict(conflict=alto.CR_DIRECT, rank_tile=16)),
    ("c3s", 32, 2, dict(conflict=alto.CR_DIRECT, rank_tile=16, block_threads=512)),
    ("unit", 20, 0, dict(conflict=alto.CR_DIRECT)),
    ("unit", 20, 2, dict(conflict=alto.CR_DIRECT)),
    ("c1", 8, 1, dict(conflict=alto.CR_DIRECT, rank_tile=4)),
    ("c2s", 32, 0, dict(conflict=alto.CR_TILE, rank_tile=8)),
    ("c2s", 64, 2, dict(conflict=alto.CR_TILE, rank_tile=16, tile_nnz=4096)),
    ("c2s", 64, 1, dict(conflict=alto.CR_RUN, rank_tile=32)),
])
def test_mttkrp_whole_mode_lds_and_rank_tiles(name, rank, mode, plan):
    X, T = built(name)
    facs = factors_for(X, rank, seed=rank + 1)
    ref = oracle_modes(X, facs)[mode]
    gf = [torch.from_numpy(f).cuda() for f in facs]
    say(f"[mttkrp] {name} R={rank} mode={mode} plan={plan}")
    got = T.mttkrp(mode, gf, plan=plan).cpu().numpy().astype(np.float64)
    check(got, ref, X, facs, mode, f"{name} R={rank} mode {mode} {plan}")


@pytest.mark.parametrize("name,rank,mode,plan", [
    # hashed tables with retention across a workgroup's tiles, FP32 and FP64 sums
    ("c2s", 16, 0, dict(conflict=alto.CR_TILE, tile_nnz=512)),
    ("c2s", 16, 2, dict(conflict=alto.CR_TILE, tile_nnz=512, accumulate=alto.ACC_F64)),
    ("c2s", 16, 2, dict(conflict=alto.CR_TILE, tile_nnz=1024, accumulate=alto.ACC_XCD_F64, block_threads=512)),
    # whole-mode tables (flushed once, after a workgroup's last tile)
    ("c3s", 32, 2, dict(conflict=alto.CR_DIRECT, rank_tile=16, tile_nnz=512)),
    ("c3s", 32, 1, dict(conflict=alto.CR_DIRECT, rank_tile=16, block_threads=512, tile_nnz=512)),
    # register runs, a 4-mode general kernel, rank tiles
    ("c2s", 16, 1, dict(conflict=alto.CR_RUN, tile_nnz=512)),
    ("c3s", 32, 0, dict(conflict=alto.CR_TILE, tile_nnz=512, rank_tile=16)),
])
def test_mttkrp_interleaved_tile_order(name, rank, mode, plan):
    """Tiles dealt round-robin to the workgroups of each XCD (short tiles, so
    that there are several per workgroup): every entry against the oracle,
    and against the same plan with contiguous stretches."""
    X, T = built(name)
    facs = factors_for(X, rank, seed=rank + 3)
    ref = oracle_modes(X, facs)[mode]
    gf = [torch.from_numpy(f).cuda() for f in facs]
    say(f"[mttkrp] interleaved {name} R={rank} mode={mode} plan={plan}")
    got = T.mttkrp(mode, gf, plan=dict(plan, tile_order=alto.ORDER_INTERLEAVED)).cpu().numpy().astype(np.float64)
    check(got, ref, X, facs, mode, f"interleaved {name} R={rank} mode {mode} {plan}")
    cont = T.mttkrp(mode, gf, plan=dict(plan, tile_order=alto.ORDER_CONTIGUOUS)).cpu().numpy().astype(np.float64)
    check(cont, ref, X, facs, mode, f"contiguous {name} R={rank} mode {mode} {plan}")
    assert rel_fro(got, cont) <= 2e-6


def test_plans_beyond_the_lds_are_rejected():
    """A hashed-table plan whose table, record staging, outboxes and static
    LDS exceed the 160 KiB a workgroup may hold is refused before any
    launch; the largest one that fits runs and matches the oracle."""
    X, T = built("c2s")
    g32 = [torch.rand(d, 32, device="cuda") for d in X.dims]
    # 1024 FP64 rows of 32 columns: 272 KiB
    with pytest.raises(alto.AltoError):
        T.mttkrp(0, g32, plan=dict(conflict=alto.CR_TILE, table_slots=1024, block_threads=256))
    # 1024 FP64 rows of 16 columns (152 KiB with keys and counts) + 8 KiB of
    # staging + 17 KiB of outboxes for 512 threads: too large
    g16 = [torch.rand(d, 16, device="cuda") for d in X.dims]
    with pytest.raises(alto.AltoError):
        T.mttkrp(1, g16, plan=dict(conflict=alto.CR_TILE, table_slots=1024, block_threads=512))
    # 512 such rows (76 KiB) fit
    facs = factors_for(X, 16, seed=17)
    gf = [torch.from_numpy(f).cuda() for f in facs]
    got = T.mttkrp(1, gf, plan=dict(conflict=alto.CR_TILE, table_slots=512, block_threads=512))
    say("[mttkrp] largest fitting table")
    check(got.cpu().numpy().astype(np.float64), oracle_modes(X, facs)[1], X, facs, 1, "largest table")


def test_whole_mode_lds_rejects_long_modes():
    X, T = built("c2s")
    gf = [torch.rand(d, 16, device="cuda") for d in X.dims]
    with pytest.raises(alto.AltoError):
        T.mttkrp(0, gf, plan=dict(conflict=alto.CR_DIRECT))
    with pytest.raises(alto.AltoError):
        T.mttkrp(0, gf, plan=dict(rank_tile=12))
    # 2048 rows x 33 FP32 columns (264 KiB) exceed the LDS; 17 columns fit
    X3, T3 = built("c3s")
    g3 = [torch.rand(d, 32, device="cuda") for d in X3.dims]
    T3.mttkrp(1, g3, plan=dict(conflict=alto.CR_DIRECT, rank_tile=16, block_threads=512))
    with pytest.raises(alto.AltoError):
        T3.mttkrp(1, g3, plan=dict(conflict=alto.CR_DIRECT, rank_tile=32))
