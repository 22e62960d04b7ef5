"""Host-side checks of the C ABI (no GPU): the library loads, exports every
declared symbol, and its planner / host extraction agree with the oracle."""

import ctypes

import numpy as np
import pytest

import oracle
import paper_2403_06348_amd as alto
from paper_2403_06348_amd import _capi


def test_library_exports_every_header_symbol():
    names = _capi.header_symbols()
    assert "alto_build" in names and "alto_mttkrp" in names and "cpd_als_sweep" in names
    L = ctypes.CDLL(_capi.LIB_PATH)
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    # every declared symbol has a ctypes signature in the binding
    assert not [n for n in names if n not in _capi.SIGNATURES], "binding lacks signatures"


@pytest.mark.parametrize(
    "dims",
    [(4, 8, 2), (64, 48, 32), (1_000_000, 500_000, 100_000), (5_000_000, 2048, 1024, 30_000), (1, 1, 7),
     (48, 64, 48, 64), (2**31, 3, 2**20 + 1, 2**31 - 1), (2**20,) * 5, (9,)],
)
def test_plan_matches_oracle(dims):
    p = alto.plan_dims(dims)
    B, nbits, _, masks = oracle.plan(dims)
    assert p["index_bits"] == B
    assert p["nbits"] == list(nbits)
    assert p["masks"] == masks
    assert p["index_words"] == (2 if B > 64 else 1)


@pytest.mark.parametrize("dims", [(4, 8, 2), (13, 1000, 7, 3), (2**25,) * 5, (2**31 - 5, 2**31, 2**31, 2**30 + 7)])
def test_host_extraction_inverts_oracle_encoding(dims):
    rng = np.random.default_rng(3)
    m = 2000
    coords = np.stack([rng.integers(0, d, m, dtype=np.int64) for d in dims])
    coords[:, 0] = np.array(dims, dtype=np.int64) - 1
    keys = oracle.encode(dims, coords)
    np.testing.assert_array_equal(alto.plan_decode_host(dims, keys), coords)


@pytest.mark.parametrize(
    "dims,status",
    [((0, 4), _capi.ERR_ARG), ((2**31 + 1, 4), _capi.ERR_ARG), ((2**31,) * 5, _capi.ERR_INDEX_BITS),
     ((2,) * 9, _capi.ERR_ARG), ((), _capi.ERR_ARG)],
)
def test_plan_argument_errors(dims, status):
    with pytest.raises(alto.AltoError) as e:
        alto.plan_dims(dims)
    assert e.value.status == status


def _header_structs():
    """Field names, in order, of every `typedef struct { ... } name;` in
    include/alto.h (array fields by name, comma lists expanded)."""
    import os
    import re

    path = os.path.join(os.path.dirname(_capi.LIB_PATH), os.pardir, "include", "alto.h")
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    out = {}
    for body, name in re.findall(r"typedef struct\s*\{(.*?)\}\s*(\w+)\s*;", text, flags=re.S):
        fields = []
        for decl in body.split(";"):
            decl = decl.strip()
            if not decl:
                continue
            # type then one or more declarators: "uint64_t a, b[4]"
            m = re.match(r"^(?:const\s+)?[\w\s\*]+?\s+(\**\w+(?:\[[^\]]*\])?(?:\s*,\s*\**\w+(?:\[[^\]]*\])?)*)$", decl)
            assert m, (name, decl)
            for d in m.group(1).split(","):
                fields.append(re.sub(r"[\*\s]|\[.*\]", "", d))
        out[name] = fields
    return out


@pytest.mark.parametrize("cname,pyname", [
    ("alto_mttkrp_plan", "MttkrpPlan"), ("alto_info_t", "Info"), ("alto_cpapr_params", "CpaprParams"),
    ("alto_serve_job", "ServeJob"), ("alto_serve_stats", "ServeStats"), ("alto_serve_done", "ServeDone"),
])
def test_binding_structs_match_header(cname, pyname):
    """Every struct the binding passes across the ABI has the header's fields
    in the header's order (a field added on one side only would shift the
    rest)."""
    hdr = _header_structs()[cname]
    py = [f for f, _ in getattr(_capi, pyname)._fields_]
    assert py == hdr, (cname, hdr, py)
