"""GPU parity of tn_distance_nodes (node-inclusive distance, the paper's
coefficient pair) against the oracle: D_nodes / D_conns bit-exact, distances
within (1e-5 + (M + 16) * 2^-24) relative, M the number of homologous genes (a
float32 sum of M non-negative terms, each a few rounded operations, is accurate
to about M + 4 unit roundoffs; the rest is two rounded quotients and a sum)."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import host, to_device
from helpers import population_from_rows

pytestmark = pytest.mark.gpu


def gpu_distance_nodes(pop, c=(1.0, 0.5)):
    import paper_2504_08339_amd as tn
    d, DN, DC = tn.distance_nodes(to_device(pop), *c)
    return host(d), host(DN), host(DC)


def _homologous(a, b):
    if a is None or b is None:
        return 0
    return len(set(a[0]) & set(b[0])) + len(set(a[1]) & set(b[1]))


def check_pairs(pop, d, DN, DC, pairs, c=(1.0, 0.5)):
    genes = {}

    def get(g):
        if g not in genes:
            genes[g] = oracle.node_genes(pop, g)
        return genes[g]

    worst = 0.0
    for i, j in pairs:
        ref, dn, dc = oracle.distance_nodes(get(i), get(j), *c)
        assert (DN[i, j], DC[i, j]) == (dn, dc), (i, j, DN[i, j], DC[i, j], dn, dc)
        if np.isnan(ref):
            assert np.isnan(d[i, j]), (i, j)
            continue
        m = _homologous(get(i), get(j))
        err = abs(float(d[i, j]) - ref)
        assert err <= (1e-5 + (m + 16) * 2.0 ** -24) * abs(ref) + 1e-7, (i, j, d[i, j], ref)
        if ref != 0:
            worst = max(worst, err / abs(ref))
    return worst


def test_xor_full_matrix():
    pop = synth.xor_population()
    d, DN, DC = gpu_distance_nodes(pop)
    check_pairs(pop, d, DN, DC, [(i, j) for i in range(pop.P) for j in range(pop.P)])


def test_control_subset_full_matrix_symmetric():
    pop = synth.control_population(P=150)
    d, DN, DC = gpu_distance_nodes(pop)
    worst = check_pairs(pop, d, DN, DC, [(i, j) for i in range(150) for j in range(150)])
    print(f"worst relative error {worst:.3g}")
    assert np.all(np.diag(d) == 0) and np.all(np.diag(DN) == 0) and np.all(np.diag(DC) == 0)
    assert np.array_equal(DN, DN.T) and np.array_equal(DC, DC.T)
    assert np.array_equal(d.view(np.uint32), d.T.view(np.uint32))


def test_control_full_size_sampled():
    """1000 x 1000 at the control population's shape; 3000 sampled pairs."""
    pop = synth.control_population()
    d, DN, DC = gpu_distance_nodes(pop)
    rng = np.random.default_rng(5)
    pairs = [tuple(p) for p in rng.integers(0, pop.P, size=(3000, 2))]
    worst = check_pairs(pop, d, DN, DC, pairs)
    print(f"worst relative error {worst:.3g}")
    assert np.array_equal(d.view(np.uint32), d.T.view(np.uint32))


def test_other_coefficients_and_mixed_attributes():
    """CPPN population: several activations per genome, disabled genes."""
    pop = synth.cppn_population(P=60)
    rng = np.random.default_rng(2)
    # vary responses, aggregations and enabled flags so every attribute term counts
    pop.node_resp[:] = rng.choice([1.0, 0.5, 2.0], size=pop.node_resp.shape).astype(np.float32)
    pop.node_agg[:] = rng.integers(0, 6, size=pop.node_agg.shape).astype(np.uint8)
    pop.conn_en[:] = rng.integers(0, 2, size=pop.conn_en.shape).astype(np.uint8)
    c = (0.7, 2.5)
    d, DN, DC = gpu_distance_nodes(pop, c)
    check_pairs(pop, d, DN, DC, [(i, j) for i in range(60) for j in range(60)], c)


def test_edge_cases():
    io = [[0, 0, 1, 0, 0], [1, 0, 1, 0, 0], [2, 0.5, 1, 2, 0]]
    genomes = [
        (io, []),                                                         # no hidden, no conns
        (io, []),
        (io + [[7, 1.0, 1, 1, 0]], [[0, 2, 0.5, 1], [0, 7, 1.0, 0]]),
        (io + [[7, -1.0, 2, 3, 4]], [[0, 2, 4.0, 0], [1, 2, 1.0, 1]]),    # act, agg, resp differ
        (io + [[7, 0, 1, 0, 0], [7, 0, 1, 0, 0]], [[0, 2, 1.0, 1]]),       # repeated node key
        (io, [[0, 2, 1.0, 1], [0, 2, 2.0, 1]]),                           # repeated marking
        ([None, io[0], None, io[1], io[2], [9, 2, 1, 0, 0]],               # holes
         [None, [9, 2, 1.0, 1], None, [0, 9, 2.0, 1]]),
        (io + [[2**30, 1, 1, 0, 0]], [[2**30, 2, 1.0, 1], [0, 2**30, 7.0, 1]]),  # large keys
        ([io[0], io[0], io[1], io[2]], [[0, 2, 1.0, 1]]),                  # repeated input key
        ([io[2], [5, 0, 1, 0, 0]], [[5, 2, 3.0, 1]]),                      # inputs missing
    ]
    pop = population_from_rows(genomes, 2, 1, N_max=6, C_max=4)
    d, DN, DC = gpu_distance_nodes(pop)
    check_pairs(pop, d, DN, DC, [(i, j) for i in range(pop.P) for j in range(pop.P)])
    for bad in (4, 5, 8):
        assert np.isnan(d[bad]).all() and (DN[bad] == -1).all() and (DC[:, bad] == -1).all()


def test_ragged_uneven():
    pop = synth.batching_population(P=70)
    d, DN, DC = gpu_distance_nodes(pop)
    rng = np.random.default_rng(9)
    pairs = [tuple(p) for p in rng.integers(0, 70, size=(300, 2))]
    check_pairs(pop, d, DN, DC, pairs)


def test_more_genomes_than_one_block():
    """P = 700 spans several 256-column blocks and odd row pairs."""
    pop = synth.control_population(P=700)
    d, DN, DC = gpu_distance_nodes(pop)
    rng = np.random.default_rng(11)
    pairs = [tuple(p) for p in rng.integers(0, 700, size=(800, 2))] + [(699, 699), (0, 699)]
    check_pairs(pop, d, DN, DC, pairs)
