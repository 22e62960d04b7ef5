"""Pins of the oracle's ALTO encoding, ordering and partitioning against values
printed in the paper (worked example, Eq. 1-3) and against invariants and
independent library routines."""

import os

import numpy as np
import pytest

import oracle
from synth import random_small_tensor

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "worked_example.txt")


def load_golden():
    g = {"coo": [], "segment": [], "prefix": []}
    with open(GOLDEN) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            tag, *rest = line.split()
            nums = [int(x) for x in rest]
            if tag in g and isinstance(g[tag], list):
                g[tag].append(nums)
            else:
                g[tag] = nums if len(nums) > 1 else nums[0]
    return g


def example():
    g = load_golden()
    coo = np.array(g["coo"], dtype=np.int64)
    coords = np.ascontiguousarray(coo[:, :3].T)
    vals = coo[:, 3].astype(np.float64)
    return g, tuple(g["dims"]), coords, vals


def key_int(k):
    return int(k[0]) | (int(k[1]) << 64)


def test_worked_example_line_length():
    g, dims, coords, _ = example()
    B, nbits, _, masks = oracle.plan(dims)
    assert B == g["line_bits"]
    keys = oracle.encode(dims, coords)
    assert all(key_int(k) < (1 << B) for k in keys)
    # masks are disjoint and cover the B index bits exactly
    acc = 0
    for m in masks:
        assert acc & m == 0
        acc |= m
    assert acc == (1 << B) - 1
    assert [bin(m).count("1") for m in masks] == list(nbits)


def test_worked_example_segments_and_intervals():
    g, dims, coords, _ = example()
    keys = oracle.encode(dims, coords)
    perm = oracle.order(keys)
    sk = keys[perm]
    starts, iv = oracle.partition(dims, sk, 2)
    assert list(starts) == [0, 3, 6]
    for l, seg in enumerate(g["segment"]):
        first, last = seg[0], seg[1]
        assert key_int(sk[starts[l]]) == first
        assert key_int(sk[starts[l + 1] - 1]) == last
        expect = np.array(seg[2:], dtype=np.uint64).reshape(3, 2)
        np.testing.assert_array_equal(iv[l], expect)


def test_worked_example_prefix_subspaces():
    g, dims, _, _ = example()
    B, _, _, _ = oracle.plan(dims)
    for pre in g["prefix"]:
        end, sub = pre[0], pre[1:]
        every = np.zeros((end + 1, 2), dtype=np.uint64)
        every[:, 0] = np.arange(end + 1, dtype=np.uint64)
        c = oracle.decode(dims, every)
        # the prefix [0-end] is exactly a box of the printed size at the origin
        assert list(c.max(axis=1) + 1) == sub
        assert int(np.prod(sub)) == end + 1
        assert len({tuple(col) for col in c.T}) == end + 1


def test_eq2_metadata_ratio_and_eq3_zmorton():
    g, dims, _, _ = example()
    B, nbits, _, _ = oracle.plan(dims)
    wb = 8
    coo_words = sum(-(-int(b) // wb) for b in nbits)
    alto_words = -(-B // wb)
    assert coo_words // alto_words == g["coo_over_alto_wb8"]
    zmorton_bits = len(dims) * int(max(nbits))
    assert (1 << zmorton_bits) // (1 << B) == g["zmorton_over_alto"]


@pytest.mark.parametrize(
    "dims,bits",
    [
        ((64, 48, 32), 6 + 6 + 5),
        ((1_000_000, 500_000, 100_000), 20 + 19 + 17),
        ((5_000_000, 2048, 1024, 30_000), 23 + 11 + 10 + 15),  # the 59-bit 4-mode workload
        ((1, 7, 1, 2), 0 + 3 + 0 + 1),
        ((2**32, 2**32, 2**32, 2**32), 128),
    ],
)
def test_eq1_index_bits(dims, bits):
    assert oracle.plan(dims)[0] == bits


def test_index_wider_than_128_bits_is_rejected():
    with pytest.raises(ValueError):
        oracle.plan((2**32, 2**32, 2**32, 2**32, 2))


def test_bit_groups_shortest_mode_first():
    # group l holds bit l of every mode with more than l bits; inside a group
    # the shorter mode sits lower, ties by mode number
    dims = (300, 40, 5000, 40, 3)
    B, nbits, pos, _ = oracle.plan(dims)
    lengths = sorted(range(len(dims)), key=lambda n: (dims[n], n))
    p = 0
    for l in range(int(max(nbits))):
        for n in lengths:
            if nbits[n] > l:
                assert pos[n, l] == p
                p += 1
    assert p == B


@pytest.mark.parametrize(
    "dims",
    [(4, 8, 2), (1, 5, 1), (13, 1000, 7, 3), (2**25, 2**25, 2**25, 2**25, 2**25), (2**32, 3, 2**31 + 1, 2**32)],
)
def test_encode_decode_round_trip(dims):
    rng = np.random.default_rng(7)
    m = 500
    coords = np.stack([rng.integers(0, d, m, dtype=np.uint64).astype(np.int64) for d in dims])
    coords[:, 0] = 0
    coords[:, 1] = np.array(dims, dtype=np.uint64).astype(np.int64) - 1
    keys = oracle.encode(dims, coords)
    np.testing.assert_array_equal(oracle.decode(dims, keys), coords)
    # the index is injective on distinct coordinates
    uniq_c = {tuple(c) for c in coords.T}
    uniq_k = {(int(a), int(b)) for a, b in keys}
    assert len(uniq_c) == len(uniq_k)


def test_encode_rejects_out_of_range():
    with pytest.raises(ValueError):
        oracle.encode((4, 8, 2), np.array([[0], [8], [0]], dtype=np.int64))
    with pytest.raises(ValueError):
        oracle.encode((4, 8, 2), np.array([[0], [-1], [0]], dtype=np.int64))


def test_order_is_numpy_stable_sort():
    X = random_small_tensor((6, 5, 7), 3000, seed=3)  # many duplicate coordinates
    keys = oracle.encode(X.dims, X.coords)
    perm = oracle.order(keys)
    expect = np.lexsort((np.arange(len(keys)), keys[:, 0], keys[:, 1]))
    np.testing.assert_array_equal(perm, expect)
    assert sorted(perm.tolist()) == list(range(len(keys)))


def test_order_128bit_keys():
    dims = (2**30, 2**30, 2**30, 2**30)
    rng = np.random.default_rng(5)
    coords = np.stack([rng.integers(0, d, 2000, dtype=np.int64) for d in dims])
    coords[:, :400] = coords[:, 400:800]  # equal keys
    keys = oracle.encode(dims, coords)
    assert np.any(keys[:, 1] != 0)
    perm = oracle.order(keys)
    np.testing.assert_array_equal(perm, np.lexsort((np.arange(2000), keys[:, 0], keys[:, 1])))


@pytest.mark.parametrize("nseg", [1, 3, 7, 64, 5000])
def test_partition_invariants(nseg):
    X = random_small_tensor((50, 9, 130), 4000, seed=11)
    keys = oracle.encode(X.dims, X.coords)
    sk = keys[oracle.order(keys)]
    starts, iv = oracle.partition(X.dims, sk, nseg)
    sizes = np.diff(starts)
    assert starts[0] == 0 and starts[-1] == len(sk)
    assert sizes.max() - sizes.min() <= 1
    c = oracle.decode(X.dims, sk)
    for l in range(nseg):
        a, b = starts[l], starts[l + 1]
        if a == b:
            assert np.all(iv[l, :, 0] == np.iinfo(np.uint64).max) and np.all(iv[l, :, 1] == 0)
            continue
        seg = c[:, a:b]
        np.testing.assert_array_equal(iv[l, :, 0], seg.min(axis=1).astype(np.uint64))
        np.testing.assert_array_equal(iv[l, :, 1], seg.max(axis=1).astype(np.uint64))
