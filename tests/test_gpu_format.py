"""GPU format generation (linearize, order, partition, de-linearize) must match
the oracle bit for bit."""

import numpy as np
import pytest

import oracle
from gpu_cases import case, say, upload

pytestmark = pytest.mark.gpu

alto = pytest.importorskip("paper_2403_06348_amd")
torch = pytest.importorskip("torch")


def oracle_sorted(X):
    keys = oracle.encode(X.dims, X.coords)
    perm = oracle.order(keys)
    return keys[perm], perm


@pytest.mark.parametrize("name", ["c1", "c2s", "c3s", "w128", "unit"])
def test_build_keys_and_values_bitexact(name):
    X = case(name)
    say(f"[format] build {name} nnz={X.nnz} dims={X.dims}")
    coords, vals = upload(X)
    T = alto.AltoTensor(X.dims, coords, vals)
    info = T.info()
    B, _, _, masks = oracle.plan(X.dims)
    assert info["index_bits"] == B and info["masks"] == masks
    keys, v = T.export()
    torch.cuda.synchronize()
    sk, perm = oracle_sorted(X)
    W = info["index_words"]
    got = keys.cpu().numpy().view(np.uint64)
    np.testing.assert_array_equal(got, sk[:, :W])
    if W == 1:
        assert not sk[:, 1].any()
    np.testing.assert_array_equal(v.cpu().numpy(), X.vals.astype(np.float32)[perm])
    # de-linearization on the GPU gives the oracle's coordinates
    dec = T.decode(keys).cpu().numpy()
    np.testing.assert_array_equal(dec, X.coords[:, perm])
    T.free()


@pytest.mark.parametrize("name,nseg", [("c1", 2), ("c1", 7), ("c2s", 1000), ("c3s", 333), ("w128", 77),
                                       ("unit", 50_010)])
def test_partition_bitexact(name, nseg):
    X = case(name)
    say(f"[format] partition {name} nseg={nseg}")
    coords, vals = upload(X)
    T = alto.AltoTensor(X.dims, coords, vals)
    starts, iv = T.partition(nseg)
    sk, _ = oracle_sorted(X)
    ost, oiv = oracle.partition(X.dims, sk, nseg)
    np.testing.assert_array_equal(starts.cpu().numpy(), ost)
    np.testing.assert_array_equal(iv.cpu().numpy().view(np.uint64), oiv)
    T.free()


def test_worked_example_on_gpu():
    from test_oracle_encoding import example, load_golden

    g, dims, coords, vals = example()
    say("[format] worked example")
    T = alto.AltoTensor(dims, torch.from_numpy(coords).cuda(), torch.from_numpy(vals.astype(np.float32)).cuda())
    keys, _ = T.export()
    k = keys.cpu().numpy().view(np.uint64)[:, 0]
    starts, iv = T.partition(2)
    st = starts.cpu().numpy()
    for l, seg in enumerate(g["segment"]):
        assert k[st[l]] == seg[0] and k[st[l + 1] - 1] == seg[1]
        np.testing.assert_array_equal(iv.cpu().numpy()[l].ravel(), np.array(seg[2:]))
    T.free()


def test_coordinate_out_of_range_is_reported():
    X = case("c1")
    coords, vals = upload(X)
    bad = coords.clone()
    bad[1, 1234] = X.dims[1]
    say("[format] out-of-range coordinate")
    with pytest.raises(alto.AltoError) as e:
        alto.AltoTensor(X.dims, bad, vals)
    assert e.value.status == alto._capi.ERR_COORD_RANGE
    assert "1234" in str(e.value)
    bad = coords.clone()
    bad[0, 7] = -1
    with pytest.raises(alto.AltoError):
        alto.AltoTensor(X.dims, bad, vals)


def test_empty_and_single_nonzero():
    say("[format] empty and single nonzero")
    dims = (5, 6, 7)
    e = torch.zeros((3, 0), dtype=torch.int64, device="cuda")
    T = alto.AltoTensor(dims, e, torch.zeros(0, dtype=torch.float32, device="cuda"))
    assert T.info()["nnz"] == 0
    f = [torch.rand(d, 8, device="cuda") for d in dims]
    out = T.mttkrp(1, f)
    assert out.shape == (6, 8) and float(out.abs().sum()) == 0.0
    T.free()
    c = torch.tensor([[4], [5], [6]], dtype=torch.int64, device="cuda")
    T = alto.AltoTensor(dims, c, torch.tensor([2.0], device="cuda"))
    keys, _ = T.export()
    ok = oracle.encode(dims, c.cpu().numpy())
    assert int(keys.cpu().numpy().view(np.uint64)[0, 0]) == int(ok[0, 0])
    T.free()
