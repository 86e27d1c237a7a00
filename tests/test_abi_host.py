"""Host-only checks of the C ABI: the library loads, exports every function the
header declares, its enums match the input encoding, and argument validation
rejects bad descriptors before anything touches a GPU."""
import ctypes
import os
import re

import pytest

from paper_2504_08339_amd import _abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER_DIR = os.path.join(ROOT, "include")


def _header_text():
    text = ""
    for f in sorted(os.listdir(HEADER_DIR)):
        if f.endswith(".h"):
            with open(os.path.join(HEADER_DIR, f)) as fh:
                text += fh.read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    return re.sub(r"//[^\n]*", " ", text)


def declared_functions():
    return sorted(set(re.findall(r"\b(tn_\w+)\s*\(", _header_text())))


def _enum_values(name):
    body = re.search(r"enum\s+" + name + r"\s*\{(.*?)\}", _header_text(), flags=re.S).group(1)
    return {k: int(v) for k, v in re.findall(r"(TN_\w+)\s*=\s*(\d+)", body)}


@pytest.fixture(scope="module")
def lib():
    return _abi.load()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 9
    for n in names:
        assert hasattr(lib, n), n
        assert n in _abi.SIGNATURES, f"{n} missing from the ctypes mirror"


def test_enums_match_encodings():
    import oracle
    import synth
    acts = _enum_values("tn_act")
    aggs = _enum_values("tn_agg")
    assert {k[len("TN_ACT_"):].lower(): v for k, v in acts.items()} == synth.ACT
    assert {k[len("TN_AGG_"):].lower(): v for k, v in aggs.items()} == synth.AGG
    assert {v: k[len("TN_ACT_"):].lower() for k, v in acts.items()} == oracle.ACT_NAMES
    assert {v: k[len("TN_AGG_"):].lower() for k, v in aggs.items()} == oracle.AGG_NAMES
    st = _enum_values("tn_genome_status")
    assert st == {"TN_CYCLE": oracle.CYCLE, "TN_DANGLING": oracle.DANGLING,
                  "TN_DUP_CONN": oracle.DUP_CONN, "TN_DUP_NODE": oracle.DUP_NODE,
                  "TN_INPUT_DST": oracle.INPUT_DST, "TN_MISSING_IO": oracle.MISSING_IO,
                  "TN_OVERSIZE": oracle.OVERSIZE, "TN_BAD_ATTR": oracle.BAD_ATTR}
    assert (_abi.TN_CYCLE, _abi.TN_BAD_ATTR) == (1, 128)


def _fake_pop(**kw):
    # Non-null dummy pointers: only host validation reads the descriptor.
    dummy = ctypes.c_void_p(0x1000)
    p = _abi.TnPopulation()
    p.P, p.n_in, p.n_out, p.N_max, p.C_max = 10, 3, 1, 16, 32
    for name in ("node_key", "node_bias", "node_resp", "node_act", "node_agg",
                 "conn_in", "conn_out", "conn_w", "conn_en"):
        setattr(p, name, ctypes.cast(dummy, dict(_abi.TnPopulation._fields_)[name]))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


@pytest.mark.parametrize("kw,code", [
    ({}, _abi.TN_OK),
    ({"P": 0}, _abi.TN_OK),
    ({"P": -1}, _abi.TN_EINVAL),
    ({"n_out": 0}, _abi.TN_EINVAL),
    ({"N_max": 0}, _abi.TN_EINVAL),
    ({"N_max": _abi.TN_MAX_NODES + 1}, _abi.TN_EUNSUPPORTED),
    ({"C_max": _abi.TN_MAX_CONNS + 1}, _abi.TN_EUNSUPPORTED),
    ({"n_in": 1000, "n_out": 100}, _abi.TN_EUNSUPPORTED),
    ({"node_key": None}, _abi.TN_EINVAL),
    ({"conn_en": None}, _abi.TN_EINVAL),
    ({"node_off": ctypes.cast(ctypes.c_void_p(0x2000), _abi.c_int64_p)}, _abi.TN_EINVAL),
])
def test_validate_population(lib, kw, code):
    p = _fake_pop(**kw)
    assert lib.tn_validate_population(ctypes.byref(p)) == code
    assert lib.tn_validate_population(None) == _abi.TN_EINVAL


def test_transformed_sizes(lib):
    p = _fake_pop()
    e = _abi.TnTransformedElems()
    assert lib.tn_transformed_size(ctypes.byref(p), ctypes.byref(e)) == _abi.TN_OK
    assert (e.node_elems, e.rowptr_elems, e.conn_elems, e.genome_elems, e.io_elems) == \
        (160, 170, 320, 10, 40)
    r = _fake_pop(node_off=ctypes.cast(ctypes.c_void_p(0x2000), _abi.c_int64_p),
                  conn_off=ctypes.cast(ctypes.c_void_p(0x3000), _abi.c_int64_p),
                  total_nodes=77, total_conns=99)
    assert lib.tn_transformed_size(ctypes.byref(r), ctypes.byref(e)) == _abi.TN_OK
    assert (e.node_elems, e.rowptr_elems, e.conn_elems) == (77, 87, 99)


def test_calls_reject_bad_arguments_without_a_gpu(lib):
    p = _fake_pop()
    tr = _abi.TnTransformed()
    assert lib.tn_forward(ctypes.byref(p), ctypes.byref(tr), None, 0, -1, None, None) == _abi.TN_EINVAL
    assert lib.tn_forward(ctypes.byref(p), ctypes.byref(tr), None, 0, 4, None, None) == _abi.TN_EINVAL
    obs = ctypes.cast(ctypes.c_void_p(0x4000), _abi.c_float_p)
    assert lib.tn_forward(ctypes.byref(p), ctypes.byref(tr), obs, 5, 4, None, None) == _abi.TN_ESHAPE
    assert lib.tn_forward(ctypes.byref(p), ctypes.byref(tr), obs, 0, 4, None, None) == _abi.TN_EINVAL
    assert lib.tn_transform(ctypes.byref(p), ctypes.byref(tr), None) == _abi.TN_EINVAL
    assert lib.tn_forward_loss(ctypes.byref(p), ctypes.byref(tr), obs, 0, 4, None, -1, 1.0, 0.0,
                               None, None, None) == _abi.TN_EINVAL
    n = ctypes.c_size_t()
    assert lib.tn_distance_workspace_size(ctypes.byref(p), ctypes.byref(n)) == _abi.TN_OK
    assert n.value > 0
    E = ctypes.cast(ctypes.c_void_p(0x5000), _abi.c_int32_p)
    assert lib.tn_distance(ctypes.byref(p), 1.0, 1.0, 0.4, None, None, E, None, None) == _abi.TN_EINVAL
    assert lib.tn_distance(ctypes.byref(p), 1.0, 1.0, 0.4, None, None, None, None, None) == _abi.TN_EINVAL
    # empty population / empty batch: nothing to do, success
    z = _fake_pop(P=0)
    assert lib.tn_forward(ctypes.byref(z), None, None, 0, 4, None, None) == _abi.TN_OK
    assert lib.tn_forward(ctypes.byref(p), ctypes.byref(tr), obs, 0, 0, None, None) == _abi.TN_OK


def test_tile_and_plan_calls_reject_bad_arguments_without_a_gpu(lib):
    p = _fake_pop()
    tr = _abi.TnTransformed()
    obs = ctypes.cast(ctypes.c_void_p(0x4000), _abi.c_float_p)
    for tile in ((7, 1, 4, 0), (_abi.TN_ENGINE_REG, 1, 4, 48), (_abi.TN_ENGINE_REG, 2, 4, 64),
                 (_abi.TN_ENGINE_LDS, 3, 4, 0), (_abi.TN_ENGINE_LDS, 1, 9, 0),
                 (_abi.TN_ENGINE_LDS, 1, 4, -1)):
        t = _abi.TnTile(*tile)
        assert lib.tn_forward_tiled(ctypes.byref(p), ctypes.byref(tr), obs, 0, 4, None,
                                    ctypes.byref(t), None) == _abi.TN_EINVAL, tile
    h = ctypes.c_void_p()
    assert lib.tn_plan_create(ctypes.byref(p), ctypes.byref(tr), 4, None, None, None) == _abi.TN_EINVAL
    assert lib.tn_plan_create(ctypes.byref(p), ctypes.byref(tr), 4, None, ctypes.byref(h),
                              None) == _abi.TN_EINVAL       # transformed arrays missing
    assert not h.value
    assert lib.tn_plan_num_buckets(None) == 0
    info = _abi.TnBucketInfo()
    assert lib.tn_plan_bucket(None, 0, ctypes.byref(info)) == _abi.TN_EINVAL
    assert lib.tn_plan_set_tile(None, 0, 1, 4) == _abi.TN_EINVAL
    for name in ("tn_plan_forward", "tn_plan_forward_buckets"):
        assert getattr(lib, name)(None, obs, 0, None, None) == _abi.TN_EINVAL
    assert lib.tn_plan_tune(None, obs, 0, None, None, None) == _abi.TN_EINVAL
    lib.tn_plan_destroy(None)


def test_status_strings(lib):
    for code in range(6):
        assert lib.tn_status_string(code).startswith(b"TN_")
    assert lib.tn_status_string(99) == b"unknown tn_status"
    assert lib.tn_version() >= 100


def test_reproduce_and_node_distance_reject_bad_arguments_without_a_gpu(lib):
    p = _fake_pop()
    nu, nz = ctypes.c_int32(), ctypes.c_int32()
    assert lib.tn_reproduce_draws(16, 32, ctypes.byref(nu), ctypes.byref(nz)) == _abi.TN_OK
    assert (nu.value, nz.value) == (16 + 7 * 16 + 2 * 32, 4 + 2 * 16 + 32)
    assert lib.tn_reproduce_draws(0, 32, ctypes.byref(nu), ctypes.byref(nz)) == _abi.TN_EINVAL
    n = ctypes.c_size_t()
    assert lib.tn_reproduce_workspace_size(-1, ctypes.byref(n)) == _abi.TN_EINVAL
    assert lib.tn_reproduce_workspace_size(100, ctypes.byref(n)) == _abi.TN_OK and n.value > 0
    good = _abi.TnMutationParams(node_add=0.2, conn_add=0.4, n_act_options=1, n_agg_options=1)
    arrays = _abi.TnPopulationArrays()
    key_out = ctypes.cast(ctypes.c_void_p(0x6000), _abi.c_int32_p)
    dummy_i = ctypes.cast(ctypes.c_void_p(0x7000), _abi.c_int32_p)
    dummy_f = ctypes.cast(ctypes.c_void_p(0x8000), _abi.c_float_p)
    ws = ctypes.c_void_p(0x9000)
    # children arrays missing
    assert lib.tn_reproduce(ctypes.byref(p), 4, dummy_i, dummy_f, dummy_f, ctypes.byref(good), 50,
                            ctypes.byref(arrays), key_out, ws, None) == _abi.TN_EINVAL
    bad = [dict(node_add=1.5), dict(conn_delete=float("nan")), dict(n_act_options=0),
           dict(n_agg_options=9), dict(act_default=256)]
    for kw in bad:
        prm = _abi.TnMutationParams(node_add=0.2, conn_add=0.4, n_act_options=1, n_agg_options=1)
        for k, v in kw.items():
            setattr(prm, k, v)
        assert lib.tn_reproduce(ctypes.byref(p), 4, dummy_i, dummy_f, dummy_f, ctypes.byref(prm),
                                50, ctypes.byref(arrays), key_out, ws, None) == _abi.TN_EINVAL, kw
    unsorted = _abi.TnMutationParams(n_act_options=2, n_agg_options=1)
    unsorted.act_options[0], unsorted.act_options[1] = 3, 1
    assert lib.tn_reproduce(ctypes.byref(p), 4, dummy_i, dummy_f, dummy_f, ctypes.byref(unsorted),
                            50, ctypes.byref(arrays), key_out, ws, None) == _abi.TN_EINVAL
    ragged = _fake_pop(node_off=ctypes.cast(ctypes.c_void_p(0x2000), _abi.c_int64_p),
                       conn_off=ctypes.cast(ctypes.c_void_p(0x3000), _abi.c_int64_p),
                       total_nodes=77, total_conns=99)
    assert lib.tn_reproduce(ctypes.byref(ragged), 4, dummy_i, dummy_f, dummy_f, ctypes.byref(good),
                            50, ctypes.byref(arrays), key_out, ws, None) == _abi.TN_EUNSUPPORTED
    assert lib.tn_distance_nodes_workspace_size(ctypes.byref(p), ctypes.byref(n)) == _abi.TN_OK
    assert n.value > 0
    E = ctypes.cast(ctypes.c_void_p(0x5000), _abi.c_int32_p)
    assert lib.tn_distance_nodes(ctypes.byref(p), 1.0, 0.5, ws, dummy_f, E, None,
                                 None) == _abi.TN_EINVAL
    assert lib.tn_distance_nodes(ctypes.byref(p), 1.0, 0.5, None, dummy_f, None, None,
                                 None) == _abi.TN_EINVAL
