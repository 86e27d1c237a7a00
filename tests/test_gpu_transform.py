"""GPU parity of tn_transform against the oracle: bit-exact status, order, level,
in-edge lists and attribute gathers, on generated, permuted, holed, ragged and
malformed populations."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import host, to_device
from helpers import population_from_rows

pytestmark = pytest.mark.gpu


def run_transform(pop):
    import paper_2504_08339_amd as tn
    dp = to_device(pop)
    tr = tn.transform(dp)
    return {k: host(getattr(tr, k)) for k in (
        "status", "n_valid", "order", "level", "row_ptr", "edge_src", "edge_row", "edge_w",
        "pos_bias", "pos_resp", "pos_fn", "io_pos")}


def blocks(pop, g):
    """(node slice, row_ptr slice start, conn slice) of genome g."""
    if pop.ragged:
        nb, ne = int(pop.node_off[g]), int(pop.node_off[g + 1])
        cb, ce = int(pop.conn_off[g]), int(pop.conn_off[g + 1])
        return slice(nb, ne), nb + g, slice(cb, ce)
    return (slice(g * pop.N_max, (g + 1) * pop.N_max), g * (pop.N_max + 1),
            slice(g * pop.C_max, (g + 1) * pop.C_max))


def compare(pop, got, genomes=None):
    want = oracle.transform_arrays(pop, genomes)
    idx = range(pop.P) if genomes is None else genomes
    nio = pop.n_in + pop.n_out
    n_checked = 0
    for a, g in enumerate(idx):
        assert got["status"][g] == want["status"][a], (g, got["status"][g], want["status"][a])
        ns, rb, cs = blocks(pop, g)
        if want["status"][a]:
            assert got["n_valid"][g] == 0
            continue
        n = want["n_valid"][a]
        assert got["n_valid"][g] == n
        order = got["order"][ns]
        assert order[:n].tolist() == want["order"][a]
        assert np.all(order[n:] == -1)
        assert got["level"][ns][:n].tolist() == want["level"][a]
        rp = got["row_ptr"][rb:rb + (ns.stop - ns.start) + 1]
        assert rp[:n + 1].tolist() == want["row_ptr"][a]
        assert np.all(rp[n + 1:] == rp[n])
        ne = want["row_ptr"][a][-1]
        assert got["edge_src"][cs][:ne].tolist() == want["edge_src"][a]
        assert got["edge_row"][cs][:ne].tolist() == want["edge_row"][a]
        ew = got["edge_w"][cs][:ne]
        assert np.array_equal(ew.view(np.uint32),
                              np.array(want["edge_w"][a], np.float32).view(np.uint32))
        assert np.all(got["edge_src"][cs][ne:] == -1) and np.all(got["edge_row"][cs][ne:] == -1)
        nr = pop.node_rows(g)
        rows = np.array(want["order"][a])
        assert np.array_equal(got["pos_bias"][ns][:n].view(np.uint32), nr["bias"][rows].view(np.uint32))
        assert np.array_equal(got["pos_resp"][ns][:n].view(np.uint32), nr["resp"][rows].view(np.uint32))
        fn = got["pos_fn"][ns][:n].astype(np.int64) & 0xffffffff
        keys = nr["key"][rows]
        exp_fn = nr["act"][rows].astype(np.int64) | (nr["agg"][rows].astype(np.int64) << 8)
        inp = keys < pop.n_in
        exp_fn[inp] |= (1 << 31) | (keys[inp].astype(np.int64) << 16)
        assert np.array_equal(fn, exp_fn)
        io = got["io_pos"][g * nio:(g + 1) * nio]
        for k in range(nio):
            assert keys[io[k]] == k
        n_checked += 1
    return n_checked


@pytest.mark.parametrize("name", ["xor", "control", "cppn", "differentiation"])
def test_generated(name):
    pop = {"xor": synth.xor_population, "control": synth.control_population,
           "cppn": synth.cppn_population,
           "differentiation": lambda: synth.differentiation_population(P=600)}[name]()
    got = run_transform(pop)
    assert compare(pop, got) == pop.P


def test_permuted_and_holed_rows():
    rng = np.random.default_rng(21)
    base = synth.control_population(P=200)
    for pop in (synth.permute_rows(base, rng), synth.insert_holes(base, rng)):
        got = run_transform(pop)
        assert compare(pop, got) == pop.P


def test_ragged_uneven_sizes():
    pop = synth.subset(synth.batching_population(P=400), range(400))
    got = run_transform(pop)
    assert compare(pop, got) == pop.P
    # the same genomes padded give the same per-genome results
    padded = synth.to_padded(pop)
    gp = run_transform(padded)
    assert compare(padded, gp) == pop.P


def test_ragged_oversize():
    pop = synth.to_ragged(synth.control_population(P=50))
    small = synth.Population(**{**pop.__dict__, "N_max": 40, "C_max": 170})
    got = run_transform(small)
    compare(small, got)
    assert (got["status"][:50] == oracle.OVERSIZE).any()


def _malformed():
    base = [[0, 0, 1, 0, 0], [1, 0, 1, 0, 0], [2, 0.5, 1, 2, 0], [7, 0, 1, 1, 0], [8, 0, 1, 3, 0]]
    cases = [
        (base, [[0, 7, 1, 1], [7, 8, 1, 1], [8, 7, 1, 1], [8, 2, 1, 1]]),   # cycle
        (base, [[0, 7, 1, 1], [7, 8, 1, 1], [8, 7, 1, 0], [8, 2, 1, 1]]),   # disabled back edge
        (base, [[0, 7, 1, 1], [7, 99, 1, 1]]),                              # dangling
        (base, [[0, 7, 1, 1], [7, 99, 1, 0]]),                              # disabled dangling
        (base, [[0, 2, 1, 1], [0, 2, 2, 1]]),                               # dup conn
        (base, [[0, 2, 1, 1], [0, 2, 2, 0]]),                               # dup conn, one disabled
        (base + [[7, 1, 1, 0, 0]], [[0, 2, 1, 1]]),                         # dup node
        (base, [[7, 1, 1, 1]]),                                             # into an input
        ([r for r in base if r[0] != 2], [[0, 7, 1, 1]]),                   # missing output
        ([r for r in base if r[0] != 0], [[1, 2, 1, 1]]),                   # missing input
        (base + [[9, 1, 1, 7, 0]], [[0, 2, 1, 1]]),                         # bad act code
        (base + [[9, 1, 1, 0, 6]], [[0, 2, 1, 1]]),                         # bad agg code
        (base, [[5, 5, 1, 1], [0, 2, 1, 1]]),                               # dangling self loop
        (base, [[7, 7, 1, 1], [0, 2, 1, 1]]),                               # self loop
        (base, []),                                                         # no connections
        ([None, None] + base, [None, [0, 2, 1, 1], None, [1, 2, -1, 1]]),  # holes
    ]
    return population_from_rows(cases, 2, 1, N_max=8, C_max=6)


def test_malformed_status_bits():
    pop = _malformed()
    got = run_transform(pop)
    compare(pop, got)
    st = got["status"][:pop.P]
    assert sorted(set(st.tolist())) == sorted(set(oracle.transform_arrays(pop)["status"]))
    assert (st != 0).sum() >= 12


def test_deterministic_reruns():
    pop = synth.batching_population(P=300)
    a = run_transform(pop)
    b = run_transform(pop)
    for k in a:
        assert np.array_equal(a[k], b[k]), k
