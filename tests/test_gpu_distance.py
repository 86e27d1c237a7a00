"""GPU parity of tn_distance against the oracle: excess / disjoint counts
bit-exact, distances within (1e-5 + (M + 8) * 2^-24) relative (a sum of M
positive float32 terms is accurate to M unit roundoffs; the rest is a handful
of rounded divisions, products and sums)."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import host, to_device
from helpers import population_from_rows

pytestmark = pytest.mark.gpu


def gpu_distance(pop, c=(1.0, 1.0, 0.4)):
    import paper_2504_08339_amd as tn
    dp = to_device(pop)
    d, E, D = tn.distance(dp, *c)
    return host(d), host(E), host(D)


def _tol(pop, i, j, ref):
    gi, gj = oracle.genome_genes(pop, i), oracle.genome_genes(pop, j)
    m = len(set(gi) & set(gj)) if gi is not None and gj is not None else 0
    return (1e-5 + (m + 8) * 2.0 ** -24) * abs(ref) + 1e-7


def check_pairs(pop, d, E, D, pairs, c=(1.0, 1.0, 0.4)):
    rd, rE, rD = oracle.distance_matrix(pop, *c, pairs=pairs)
    for (i, j), a, e, dd in zip(pairs, rd, rE, rD):
        assert (E[i, j], D[i, j]) == (e, dd), (i, j)
        if np.isnan(a):
            assert np.isnan(d[i, j])
        else:
            assert abs(d[i, j] - a) <= _tol(pop, i, j, a), (i, j, d[i, j], a)


def test_xor_full_matrix():
    pop = synth.xor_population()
    d, E, D = gpu_distance(pop)
    pairs = [(i, j) for i in range(pop.P) for j in range(pop.P)]
    check_pairs(pop, d, E, D, pairs)


def test_control_subset_full_matrix_and_symmetry():
    pop = synth.control_population(P=150)
    d, E, D = gpu_distance(pop)
    check_pairs(pop, d, E, D, [(i, j) for i in range(150) for j in range(150)])
    assert np.array_equal(E, E.T) and np.array_equal(D, D.T)
    assert np.array_equal(d.view(np.uint32), d.T.view(np.uint32))


def test_control_full_size_sampled():
    """1000 x 1000 matrix in the benchmark's launch configuration; 3000 sampled
    pairs against the oracle, plus whole-matrix invariants."""
    pop = synth.control_population()
    d, E, D = gpu_distance(pop)
    rng = np.random.default_rng(3)
    pairs = [tuple(p) for p in rng.integers(0, pop.P, size=(3000, 2))]
    check_pairs(pop, d, E, D, pairs)
    assert np.all(np.diag(d) == 0) and np.all(np.diag(E) == 0)
    assert np.array_equal(E, E.T) and np.array_equal(d.view(np.uint32), d.T.view(np.uint32))


def test_other_coefficients_and_disabled_genes():
    pop = synth.cppn_population(P=60)
    c = (0.7, 2.5, 1.3)
    d, E, D = gpu_distance(pop, c)
    check_pairs(pop, d, E, D, [(i, j) for i in range(60) for j in range(60)], c)


def test_edge_cases():
    nodes = [[0, 0, 1, 0, 0]]
    genomes = [
        (nodes, []),                                              # empty
        (nodes, []),                                              # empty
        (nodes, [[0, 3, 0.5, 1], [1, 3, 1.0, 0], [2, 3, -1.0, 1]]),
        (nodes, [[2, 3, 4.0, 1], [0, 3, 0.0, 0]]),
        (nodes, [[0, 3, 1.0, 1], [0, 3, 2.0, 1]]),                # repeated marking
        (nodes, [None, [5, 9, 1.0, 1], None, [1, 3, 2.0, 1]]),   # holes
        (nodes, [[2**30, 2**30 + 1, 1.0, 1], [0, 3, 7.0, 1]]),   # large keys
    ]
    pop = population_from_rows(genomes, 0, 1, C_max=4)
    d, E, D = gpu_distance(pop)
    check_pairs(pop, d, E, D, [(i, j) for i in range(pop.P) for j in range(pop.P)])
    assert np.isnan(d[4]).all() and (E[4] == -1).all()


def test_ragged_uneven():
    pop = synth.batching_population(P=70)
    d, E, D = gpu_distance(pop)
    rng = np.random.default_rng(8)
    pairs = [tuple(p) for p in rng.integers(0, 70, size=(300, 2))]
    check_pairs(pop, d, E, D, pairs)
