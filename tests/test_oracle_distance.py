"""Pins of the oracle's compatibility distance.

Checked against hand-counted pairs (tests/golden/distance_pairs.json), an
independent two-pointer merge over sorted gene lists written here, and the
properties the definition implies (identity, symmetry, disjoint gene sets).
"""
import numpy as np
import pytest

import oracle
import synth
from helpers import load_golden, population_from_rows

GOLD = load_golden("distance_pairs.json")


def _pair_pop(g1, g2):
    nodes = [[0, 0, 1, 0, 0]]
    return population_from_rows([(nodes, g1), (nodes, g2)], 0, 0,
                                C_max=max(1, len(g1), len(g2)))


@pytest.mark.parametrize("case", GOLD["cases"], ids=[c["name"] for c in GOLD["cases"]])
def test_hand_counted(case):
    pop = _pair_pop(case["g1"], case["g2"])
    d, E, D = oracle.distance(oracle.genome_genes(pop, 0), oracle.genome_genes(pop, 1),
                              GOLD["c1"], GOLD["c2"], GOLD["c3"])
    assert (E, D) == (case["E"], case["D"])
    assert d == pytest.approx(case["delta"], rel=1e-6, abs=1e-7)
    d2, E2, D2 = oracle.distance(oracle.genome_genes(pop, 1), oracle.genome_genes(pop, 0),
                                 GOLD["c1"], GOLD["c2"], GOLD["c3"])
    assert (E2, D2, d2) == (E, D, d)


def _merge_counts(pop, i, j):
    """Two-pointer merge over lexicographically sorted markings."""
    def genes(g):
        rows = [(int(a), int(b), float(w)) for a, b, w in
                zip(pop.conn_in[g], pop.conn_out[g], pop.conn_w[g]) if a >= 0 and b >= 0]
        return sorted(rows)
    A, B = genes(i), genes(j)
    a = b = 0
    m = 0
    wsum = 0.0
    only_a, only_b = [], []
    while a < len(A) and b < len(B):
        ka, kb = A[a][:2], B[b][:2]
        if ka == kb:
            m += 1
            wsum += abs(A[a][2] - B[b][2])
            a += 1
            b += 1
        elif ka < kb:
            only_a.append(ka)
            a += 1
        else:
            only_b.append(kb)
            b += 1
    only_a += [g[:2] for g in A[a:]]
    only_b += [g[:2] for g in B[b:]]
    if not A and not B:
        return 0, 0, 0.0, 0
    if A and B:
        lim = min(A[-1][:2], B[-1][:2])
        E = sum(1 for k in only_a + only_b if k > lim)
    else:
        E = len(only_a) + len(only_b)
    D = len(only_a) + len(only_b) - E
    return E, D, (wsum / m if m else 0.0), max(len(A), len(B))


def test_against_independent_merge():
    pop = synth.control_population(P=40)
    dist, E, D = oracle.distance_matrix(pop)
    for i in range(pop.P):
        for j in range(pop.P):
            e, d, wbar, n = _merge_counts(pop, i, j)
            assert (E[i, j], D[i, j]) == (e, d)
            assert dist[i, j] == pytest.approx(e / n + d / n + 0.4 * wbar, rel=1e-12)


def test_properties():
    pop = synth.control_population(P=30)
    dist, E, D = oracle.distance_matrix(pop)
    assert np.all(np.diag(dist) == 0) and np.all(np.diag(E) == 0) and np.all(np.diag(D) == 0)
    assert np.array_equal(dist, dist.T) and np.array_equal(E, E.T) and np.array_equal(D, D.T)
    assert np.all(dist >= 0)


def test_disjoint_gene_sets():
    rng = np.random.default_rng(4)
    for _ in range(50):
        keys = rng.choice(400, size=rng.integers(2, 40), replace=False)
        split = rng.integers(1, len(keys))
        g1 = [[int(k) // 20, 100 + int(k) % 20, float(rng.standard_normal()), 1] for k in keys[:split]]
        g2 = [[int(k) // 20, 100 + int(k) % 20, float(rng.standard_normal()), 0] for k in keys[split:]]
        pop = _pair_pop(g1, g2)
        d, E, D = oracle.distance(oracle.genome_genes(pop, 0), oracle.genome_genes(pop, 1))
        assert E + D == len(g1) + len(g2)
        assert d == pytest.approx((E + D) / max(len(g1), len(g2)), rel=1e-12)


def test_duplicate_marking_is_nan():
    pop = _pair_pop([[0, 1, 1.0, 1], [0, 1, 2.0, 0]], [[0, 1, 1.0, 1]])
    d, E, D = oracle.distance(oracle.genome_genes(pop, 0), oracle.genome_genes(pop, 1))
    assert np.isnan(d) and E == -1 and D == -1
