"""Pins of the oracle's decoding and transformation (TensorNEAT Section 3.3).

The oracle is checked against things it does not compute itself: brute-force
enumeration of every 3-node graph, the longest-path closed form of the
level-synchronous order, structural invariants of the in-edge lists, and
hand-built malformed genomes whose status bits are known by construction.
"""
import itertools

import numpy as np
import pytest

import oracle
import synth
from helpers import population_from_rows

KEYS = (10, 11, 12)
PAIRS = [(a, b) for a in range(3) for b in range(3) if a != b]


def _brute_levels(enabled_pairs):
    """Longest enabled path ending at each node, by enumerating node sequences."""
    level = {v: 0 for v in range(3)}
    for length in (2, 3):
        for seq in itertools.permutations(range(3), length):
            if all((seq[i], seq[i + 1]) in enabled_pairs for i in range(length - 1)):
                level[seq[-1]] = max(level[seq[-1]], length - 1)
    return level


def _linear_extensions(enabled_pairs):
    return [p for p in itertools.permutations(range(3))
            if all(p.index(a) < p.index(b) for a, b in enabled_pairs)]


@pytest.mark.parametrize("row_perm", list(itertools.permutations(range(3))))
def test_brute_force_three_node_graphs(row_perm):
    """All 3^6 graphs on 3 nodes (each ordered pair absent / enabled / disabled),
    under every assignment of nodes to rows."""
    genomes, meta = [], []
    for states in itertools.product(range(3), repeat=6):
        nodes = [None] * 3
        for v in range(3):
            nodes[row_perm[v]] = [KEYS[v], 0.0, 1.0, 0, 0]
        conns = []
        enabled = set()
        for (a, b), s in zip(PAIRS, states):
            if s == 0:
                continue
            conns.append([KEYS[a], KEYS[b], 1.0, 1 if s == 1 else 0])
            if s == 1:
                enabled.add((a, b))
        genomes.append((nodes, conns))
        meta.append(enabled)
    pop = population_from_rows(genomes, 0, 0, N_max=3, C_max=6)
    n_cyclic = 0
    for g, enabled in enumerate(meta):
        tr = oracle.transform(oracle.decode(pop, g))
        exts = _linear_extensions(enabled)
        if not exts:
            n_cyclic += 1
            assert tr.status == oracle.CYCLE
            continue
        assert tr.status == 0
        order = [KEYS.index(k) for k in tr.order]
        assert tuple(order) in exts
        lv = _brute_levels(enabled)
        closed = sorted(range(3), key=lambda v: (lv[v], row_perm[v]))
        assert order == closed
        assert all(tr.level[KEYS[v]] == lv[v] for v in range(3))
        # disabled edges have no effect: same genome with them removed
        only_enabled = [c for c in genomes[g][1] if c[3] == 1]
        pop2 = population_from_rows([(genomes[g][0], only_enabled)], 0, 0, N_max=3, C_max=6)
        assert oracle.transform(oracle.decode(pop2, 0)).order == tr.order
    # 2-cycles and 3-cycles among the 729 graphs
    assert n_cyclic > 0


def test_self_loop():
    nodes = [[0, 0, 1, 0, 0], [1, 0, 1, 0, 0], [5, 0, 1, 0, 0]]
    on = population_from_rows([(nodes, [[0, 1, 1.0, 1], [5, 5, 1.0, 1]])], 1, 1)
    off = population_from_rows([(nodes, [[0, 1, 1.0, 1], [5, 5, 1.0, 0]])], 1, 1)
    assert oracle.transform(oracle.decode(on, 0)).status == oracle.CYCLE
    assert oracle.transform(oracle.decode(off, 0)).status == 0


def _check_structure(pop, g, arr, a):
    """Structural invariants of one genome's transformed arrays."""
    gen = oracle.decode(pop, g)
    n = arr["n_valid"][a]
    order, level = arr["order"][a], arr["level"][a]
    rp, es, er, ew = (arr["row_ptr"][a], arr["edge_src"][a], arr["edge_row"][a],
                      arr["edge_w"][a])
    keys = pop.node_key[g]
    # every valid node exactly once
    assert sorted(order) == sorted(int(r) for r in np.flatnonzero(keys >= 0))
    assert n == len(order)
    # in-edges of position p: exactly the enabled rows ending at that node
    enabled_rows = sorted(c.row for c in gen.conns if c.enabled)
    assert sorted(er) == enabled_rows
    assert rp[0] == 0 and rp[-1] == len(er)
    for p in range(n):
        rows = er[rp[p]:rp[p + 1]]
        assert rows == sorted(rows)
        for e in range(rp[p], rp[p + 1]):
            r = er[e]
            assert pop.conn_out[g, r] == keys[order[p]]
            assert pop.conn_in[g, r] == keys[order[es[e]]]
            assert es[e] < p
            assert ew[e] == pop.conn_w[g, r]
        # longest-path characterisation of the level
        if rp[p] == rp[p + 1]:
            assert level[p] == 0
        else:
            assert level[p] == 1 + max(level[es[e]] for e in range(rp[p], rp[p + 1]))
    # positions sorted by (level, node row)
    assert [(level[p], order[p]) for p in range(n)] == sorted(zip(level, order))


@pytest.mark.parametrize("maker", [synth.xor_population,
                                   lambda: synth.control_population(P=120),
                                   lambda: synth.cppn_population(P=120)])
def test_structure_generated(maker):
    pop = maker()
    arr = oracle.transform_arrays(pop)
    assert all(s == 0 for s in arr["status"])
    for g in range(pop.P):
        _check_structure(pop, g, arr, g)


def test_holes_and_row_permutation_keep_key_order():
    rng = np.random.default_rng(7)
    pop = synth.control_population(P=40)
    holes = synth.insert_holes(pop, rng)
    base = oracle.transform_population(pop)
    for g, (gen, tr) in enumerate(base):
        gh = oracle.decode(holes, g)
        th = oracle.transform(gh)
        assert th.order == tr.order            # relative row order unchanged
        assert th.level == tr.level
    perm = synth.permute_rows(pop, rng)
    for g, (gen, tr) in enumerate(base):
        tp = oracle.transform(oracle.decode(perm, g))
        assert tp.level == tr.level            # levels are row independent
        arr = oracle.transform_arrays(perm, [g])
        _check_structure(perm, g, arr, 0)


def _one(nodes, conns, n_in=2, n_out=1):
    pop = population_from_rows([(nodes, conns)], n_in, n_out)
    return oracle.transform(oracle.decode(pop, 0)).status


BASE_NODES = [[0, 0, 1, 0, 0], [1, 0, 1, 0, 0], [2, 0, 1, 0, 0], [7, 0, 1, 0, 0], [8, 0, 1, 0, 0]]


@pytest.mark.parametrize("nodes,conns,expected", [
    (BASE_NODES, [[0, 7, 1, 1], [7, 8, 1, 1], [8, 7, 1, 1], [8, 2, 1, 1]], oracle.CYCLE),
    (BASE_NODES, [[0, 7, 1, 1], [7, 8, 1, 1], [8, 7, 1, 0], [8, 2, 1, 1]], 0),
    (BASE_NODES, [[0, 7, 1, 1], [7, 99, 1, 1]], oracle.DANGLING),
    (BASE_NODES, [[0, 7, 1, 1], [7, 99, 1, 0]], 0),
    (BASE_NODES, [[0, 2, 1, 1], [0, 2, 2, 1]], oracle.DUP_CONN),
    (BASE_NODES, [[0, 2, 1, 1], [0, 2, 2, 0]], oracle.DUP_CONN),
    (BASE_NODES + [[7, 1, 1, 0, 0]], [[0, 2, 1, 1]], oracle.DUP_NODE),
    (BASE_NODES, [[7, 1, 1, 1]], oracle.INPUT_DST),
    (BASE_NODES, [[7, 1, 1, 0]], 0),
    ([r for r in BASE_NODES if r[0] != 2], [[0, 7, 1, 1]], oracle.MISSING_IO),
    ([r for r in BASE_NODES if r[0] != 0], [[1, 2, 1, 1]], oracle.MISSING_IO),
    (BASE_NODES, [[0, 7, 1, 1], [7, 0, 1, 1]], oracle.INPUT_DST),  # CYCLE is only looked for when no other bit is set
    (BASE_NODES + [[8, 1, 1, 0, 0]], [[0, 2, 1, 1], [0, 2, 1, 1], [2, 55, 1, 1]],
     oracle.DUP_NODE | oracle.DUP_CONN | oracle.DANGLING),
    (BASE_NODES + [[9, 1, 1, 7, 0]], [[0, 2, 1, 1]], oracle.BAD_ATTR),
    (BASE_NODES + [[9, 1, 1, 0, 6]], [[0, 2, 1, 1]], oracle.BAD_ATTR),
])
def test_status_bits(nodes, conns, expected):
    assert _one(nodes, conns) == expected


def test_empty_rows_anywhere_and_negative_keys():
    nodes = [None, [0, 0, 1, 0, 0], None, [1, 0, 1, 0, 0], [2, 0, 1, 0, 0], None]
    conns = [None, [0, 2, 1, 1], [-1, 2, 5, 1], [1, -1, 5, 1], None, [1, 2, 1, 1]]
    pop = population_from_rows([(nodes, conns)], 2, 1, N_max=6, C_max=6)
    gen = oracle.decode(pop, 0)
    assert sorted(gen.nodes) == [0, 1, 2]
    assert [c.row for c in gen.conns] == [1, 5]
    tr = oracle.transform(gen)
    assert tr.status == 0 and tr.order == [0, 1, 2]


def test_oversize_ragged():
    pop = synth.to_ragged(synth.xor_population(P=5))
    small = synth.Population(**{**pop.__dict__, "N_max": 3})
    st = [oracle.transform(oracle.decode(small, g)).status for g in range(5)]
    assert all(s == oracle.OVERSIZE for s in st)
