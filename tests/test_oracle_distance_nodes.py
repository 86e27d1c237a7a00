"""Pins of the oracle's node-inclusive distance (the paper's coefficient pair,
Appendix A; formula reading in oracle/compat.py).

Hand-worked pairs (tests/golden/distance_nodes_pairs.json); reduction to the
connection-gene NEAT distance (pinned on its own) when two genomes hold the
same node genes and agree on every enabled flag; invariants (identity,
symmetry, hidden-key relabelling, row permutation); planted mistakes."""
import numpy as np
import pytest

import oracle
import oracle.compat as oc
import synth
from helpers import load_golden, population_from_rows

GOLD = load_golden("distance_nodes_pairs.json")


def _pop(names):
    gs = [GOLD["genomes"][n] for n in names]
    return population_from_rows([(g["nodes"], g["conns"]) for g in gs], 2, 1, N_max=6, C_max=6)


@pytest.mark.parametrize("case", GOLD["pairs"], ids=lambda c: f"{c['a']}-{c['b']}")
def test_hand_pairs(case):
    pop = _pop([case["a"], case["b"]])
    d, dn, dc = oracle.distance_nodes(oracle.node_genes(pop, 0), oracle.node_genes(pop, 1))
    assert d == pytest.approx(case["delta"], abs=1e-12)
    assert (dn, dc) == (case["d_nodes"], case["d_conns"])


def test_reduces_to_neat_distance_on_shared_nodes():
    """Same node genes, equal enabled flags on shared markings: delta equals
    the connection-gene NEAT distance with c1 = c2 = c_d, c3 = c_h * M / N."""
    pop = synth.control_population(P=20)
    rng = np.random.default_rng(3)
    pairs = []
    for g in range(pop.P):
        a = synth.subset(pop, [g, g])
        valid = np.flatnonzero(a.conn_in[1] >= 0)
        drop = rng.choice(valid, size=len(valid) // 4, replace=False)
        a.conn_in[1, drop] = -1
        a.conn_out[1, drop] = -1
        a.conn_w[1] = a.conn_w[1] + rng.standard_normal(a.C_max).astype(np.float32)
        pairs.append(a)
    checked = 0
    for a in pairs:
        ga, gb = oracle.node_genes(a, 0), oracle.node_genes(a, 1)
        assert ga[0] == gb[0]
        d, dn, dc = oracle.distance_nodes(ga, gb, 1.0, 0.5)
        ca, cb = oracle.genome_genes(a, 0), oracle.genome_genes(a, 1)
        M = len(set(ca) & set(cb))
        N = max(len(ca), len(cb))
        neat, E, D = oracle.distance(ca, cb, 1.0, 1.0, 0.5 * M / N)
        assert dn == 0 and dc == E + D
        assert d == pytest.approx(neat, rel=1e-12, abs=1e-12)
        checked += 1
    assert checked == pop.P


def test_identity_symmetry_relabel_permutation():
    pop = synth.control_population(P=12)
    d, dn, dc = oracle.distance_nodes_matrix(pop)
    assert np.all(np.diag(d) == 0) and np.all(np.diag(dn) == 0) and np.all(np.diag(dc) == 0)
    np.testing.assert_allclose(d, d.T, rtol=1e-15, atol=0)
    assert np.array_equal(dn, dn.T) and np.array_equal(dc, dc.T)
    assert (d[~np.eye(pop.P, dtype=bool)] > 0).all()
    rel = synth.subset(pop, range(pop.P))
    n_io = pop.n_in + pop.n_out
    for arr in (rel.node_key, rel.conn_in, rel.conn_out):
        hid = arr >= n_io
        arr[hid] = 3 * arr[hid] + 11
    d2, dn2, dc2 = oracle.distance_nodes_matrix(rel)
    np.testing.assert_allclose(d2, d, rtol=1e-12, atol=0)
    assert np.array_equal(dn2, dn) and np.array_equal(dc2, dc)
    perm = synth.permute_rows(pop, np.random.default_rng(1))
    d3, dn3, dc3 = oracle.distance_nodes_matrix(perm)
    np.testing.assert_allclose(d3, d, rtol=1e-12, atol=0)
    assert np.array_equal(dn3, dn) and np.array_equal(dc3, dc)


def test_repeated_key_has_no_gene_set():
    pop = _pop(["g1", "g2"])
    pop.node_key[0, 3] = 2
    d, dn, dc = oracle.distance_nodes(oracle.node_genes(pop, 0), oracle.node_genes(pop, 1))
    assert np.isnan(d) and dn == dc == -1


# ---- planted mistakes ---------------------------------------------------------

def _fails(fn, *a):
    try:
        fn(*a)
    except AssertionError:
        return True
    return False


def test_planted_enabled_flag_ignored(monkeypatch):
    monkeypatch.setattr(oc, "_conn_attr_distance", lambda p, q: abs(p[0] - q[0]))
    assert _fails(test_hand_pairs, GOLD["pairs"][0])


def test_planted_inputs_counted(monkeypatch):
    orig = oc.node_genes

    def wrong(pop, g):
        r = orig(pop, g)
        if r is not None:
            for k in range(pop.n_in):
                r[0][k] = (0.0, 1.0, 0, 0)
        return r
    monkeypatch.setattr(oc, "node_genes", wrong)
    monkeypatch.setattr(oracle, "node_genes", wrong)
    assert _fails(test_hand_pairs, GOLD["pairs"][0])


def test_planted_scaled_result(monkeypatch):
    orig = oc.distance_nodes

    def wrong(a, b, c_d=1.0, c_h=0.5):
        d, dn, dc = orig(a, b, c_d, c_h)
        return d * 0.9, dn, dc
    monkeypatch.setattr(oracle, "distance_nodes", wrong)
    assert _fails(test_reduces_to_neat_distance_on_shared_nodes)
