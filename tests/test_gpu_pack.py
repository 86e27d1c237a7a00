"""tn_pack_paper_layout through the C ABI: the paper's NaN-padded float tensors
(Section 3.1) become the structure-of-arrays population bit for bit; NaN rows
anywhere become holes; rows breaking the encoding's rules are rejected."""
import numpy as np
import pytest
import torch

import paper_2504_08339_amd as tn
import synth
from gpu_util import FIELDS, host, tensor

pytestmark = pytest.mark.gpu


def _pack(pop, **kw):
    PN, PC = synth.to_paper_layout(pop)
    return tn.pack_paper_layout(tensor(PN), tensor(PC), pop.n_in, pop.n_out, **kw)


def _same(dp, pop):
    for k in FIELDS:
        got = host(dp.t[k])
        want = getattr(pop, k)
        # empty rows: key / markings -1, the other fields 0
        assert got.dtype == want.dtype, k
        assert np.array_equal(got.view(np.uint8), want.view(np.uint8)), k


@pytest.mark.parametrize("make", [
    lambda: synth.xor_population(P=150),
    lambda: synth.control_population(P=200),
    lambda: synth.insert_holes(synth.control_population(P=120), np.random.default_rng(3)),
    lambda: synth.permute_rows(synth.cppn_population(P=90), np.random.default_rng(4)),
], ids=["xor", "control", "control_holes", "cppn_permuted"])
def test_pack_equals_soa_bitwise(make):
    pop = make()
    dp = _pack(pop)
    _same(dp, pop)
    # the packed population transforms and evaluates exactly as the SoA one
    from gpu_util import to_device
    obs = tensor(synth.normal_obs(pop.P, 70, pop.n_in, 5))
    ref = to_device(pop)
    y0 = tn.forward(ref, tn.transform(ref), obs)
    y1 = tn.forward(dp, tn.transform(dp), obs)
    assert torch.equal(y0.view(torch.int32), y1.view(torch.int32))


def test_nan_rows_anywhere_become_holes():
    pop = synth.control_population(P=40)
    PN, PC = synth.to_paper_layout(pop)
    rng = np.random.default_rng(8)
    # a NaN first column empties a row whatever its other columns hold
    for g in range(pop.P):
        r = int(rng.integers(pop.N_max))
        PN[g, r, 0] = np.nan
        PN[g, r, 1:] = 7.0
        c = int(rng.integers(pop.C_max))
        PC[g, c, 0] = np.nan
        PC[g, c, 1:] = 3.0
        pop.node_key[g, r] = -1
        pop.node_bias[g, r] = pop.node_resp[g, r] = 0
        pop.node_act[g, r] = pop.node_agg[g, r] = 0
        pop.conn_in[g, c] = pop.conn_out[g, c] = -1
        pop.conn_w[g, c] = 0
        pop.conn_en[g, c] = 0
    dp = tn.pack_paper_layout(tensor(PN), tensor(PC), pop.n_in, pop.n_out)
    _same(dp, pop)


@pytest.mark.parametrize("where,col,value,bit", [
    ("node", 0, 3.5, tn.TN_PACK_NODE_KEY),
    ("node", 0, 2.0 ** 24, tn.TN_PACK_NODE_KEY),
    ("node", 0, -2.0, tn.TN_PACK_NODE_KEY),
    ("node", 0, np.inf, tn.TN_PACK_NODE_KEY),
    ("node", 3, 1.5, tn.TN_PACK_NODE_CODE),
    ("node", 4, 300.0, tn.TN_PACK_NODE_CODE),
    ("node", 3, np.nan, tn.TN_PACK_NODE_CODE),
    ("conn", 0, 0.25, tn.TN_PACK_CONN_KEY),
    ("conn", 1, np.nan, tn.TN_PACK_CONN_KEY),
    ("conn", 1, 2.0 ** 24 + 2, tn.TN_PACK_CONN_KEY),
    ("conn", 2, 0.5, tn.TN_PACK_CONN_FLAG),
    ("conn", 2, 2.0, tn.TN_PACK_CONN_FLAG),
])
def test_bad_rows_rejected(where, col, value, bit):
    pop = synth.control_population(P=12)
    PN, PC = synth.to_paper_layout(pop)
    g = 5
    if where == "node":
        r = int(np.flatnonzero(pop.node_key[g] >= 0)[-1])
        PN[g, r, col] = value
    else:
        r = int(np.flatnonzero(pop.conn_in[g] >= 0)[-1])
        PC[g, r, col] = value
    dp, err, rc = tn.pack_paper_layout(tensor(PN), tensor(PC), pop.n_in, pop.n_out,
                                       return_errors=True)
    assert rc == 1  # TN_EINVAL
    e = host(err)
    assert e[g] == bit and np.count_nonzero(e) == 1
    # the bad row is written empty, every other row converted
    if where == "node":
        pop.node_key[g, r] = -1
        pop.node_bias[g, r] = pop.node_resp[g, r] = 0
        pop.node_act[g, r] = pop.node_agg[g, r] = 0
    else:
        pop.conn_in[g, r] = pop.conn_out[g, r] = -1
        pop.conn_w[g, r] = 0
        pop.conn_en[g, r] = 0
    _same(dp, pop)
    with pytest.raises(tn.TNError):
        tn.pack_paper_layout(tensor(PN), tensor(PC), pop.n_in, pop.n_out)


def test_largest_exact_key_and_empty_population():
    pop = synth.xor_population(P=3)
    PN, PC = synth.to_paper_layout(pop)
    # the largest key below 2^24 is accepted (a hidden node no edge uses)
    r = int(np.flatnonzero(pop.node_key[1] < 0)[0])
    PN[1, r] = [2.0 ** 24 - 1, 0.5, 1.0, 1.0, 0.0]
    pop.node_key[1, r] = 2 ** 24 - 1
    pop.node_bias[1, r], pop.node_resp[1, r], pop.node_act[1, r], pop.node_agg[1, r] = 0.5, 1, 1, 0
    _same(tn.pack_paper_layout(tensor(PN), tensor(PC), pop.n_in, pop.n_out), pop)
    z = tn.pack_paper_layout(tensor(PN[:0]), tensor(PC[:0]), 3, 1)
    assert z.P == 0
