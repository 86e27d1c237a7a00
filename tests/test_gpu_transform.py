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


FIELDS = ("status", "n_valid", "order", "level", "row_ptr", "edge_src", "edge_row", "edge_w",
          "pos_bias", "pos_resp", "pos_fn", "io_pos", "pos_row", "n_rows", "prog_node",
          "prog_edge", "prog_rows", "prog_rec")


def run_transform(pop):
    import paper_2504_08339_amd as tn
    dp = to_device(pop)
    tr = tn.transform(dp)
    return {k: host(getattr(tr, k)) for k in FIELDS}


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


def test_large_ragged_population_by_size_class():
    """A ragged population of 2200 uneven genomes (the library transforms one
    of at least 2048 genomes in launches by size class): genomes appended
    with hole connection rows, so that their connection rows and not their
    node rows decide the class, and a node capacity below the largest genomes
    (those are OVERSIZE). Statuses of every genome; every field bit-exact
    against the oracle on the padded genomes, on both sides of each class
    bound and on a random sample."""
    base = synth.batching_population(P=2200)
    rng = np.random.default_rng(77)
    padded_ids = rng.choice(2200, size=40, replace=False)
    nb, cb, n_off, c_off = [], [], [0], [0]
    for g in range(base.P):
        n = base.node_rows(g)
        c = {k: v.copy() for k, v in base.conn_rows(g).items()}
        if g in padded_ids:
            extra = int(rng.integers(300, 700))   # holes: rows with in = out = -1
            c = {k: np.concatenate([v, np.full(extra, -1 if k in ("in", "out") else 0, v.dtype)])
                 for k, v in c.items()}
        nb.append(n)
        cb.append(c)
        n_off.append(n_off[-1] + n["key"].shape[0])
        c_off.append(c_off[-1] + c["in"].shape[0])
    cat = lambda bl, k: np.concatenate([b[k] for b in bl])
    rows = np.diff(n_off)
    N_cap = int(np.sort(rows)[-5])                # the four largest genomes exceed it
    pop = synth.Population(base.n_in, base.n_out, N_cap, int(np.diff(c_off).max()),
                           cat(nb, "key"), cat(nb, "bias"), cat(nb, "resp"), cat(nb, "act"),
                           cat(nb, "agg"), cat(cb, "in"), cat(cb, "out"), cat(cb, "w"), cat(cb, "en"),
                           np.array(n_off, np.int64), np.array(c_off, np.int64))
    got = run_transform(pop)
    over = rows > N_cap
    assert over.sum() == 4
    assert (got["status"][:pop.P][over] == oracle.OVERSIZE).all()
    assert (got["status"][:pop.P][~over] == 0).all()
    crows = np.diff(c_off)
    near = [g for g in range(pop.P) if any(abs(int(rows[g]) - b) <= 2 for b in (96, 192, 320, 400))
            or any(abs(int(crows[g]) - b) <= 8 for b in (384, 768, 1280, 1600))]
    sample = sorted(set(padded_ids.tolist()) | set(near[:120]) |
                    set(rng.choice(pop.P, size=120, replace=False).tolist()) |
                    set(np.flatnonzero(over).tolist()))
    assert compare(pop, got, sample) == len(sample) - int(over.sum())
    for g in sample:
        if not over[g]:
            _check_rows(pop, got, g)


def _large_defective(rng):
    """The 60 largest genomes of a 400-genome batching population, padded with
    room for extra rows, with defects injected into the first six: a two-node
    cycle, a duplicated connection, a dangling enabled connection, an enabled
    connection into an input, a long cycle closing a path of several levels,
    and a duplicated node key; the rest stay valid."""
    base = synth.batching_population(P=400)
    sizes = np.diff(base.node_off)
    big = synth.subset(base, np.argsort(-sizes, kind="stable")[:60])
    pop = synth.to_padded(big, N_max=big.N_max + 2, C_max=big.C_max + 4)

    def add_conn(g, a, b, en=1):
        r = int(np.flatnonzero(pop.conn_in[g] < 0)[0])
        pop.conn_in[g, r], pop.conn_out[g, r] = a, b
        pop.conn_w[g, r], pop.conn_en[g, r] = 0.5, en

    def edges(g):
        m = (pop.conn_in[g] >= 0) & (pop.conn_en[g] > 0)
        return list(zip(pop.conn_in[g][m].tolist(), pop.conn_out[g][m].tolist()))

    io = pop.n_in + pop.n_out
    hidden_edges = lambda g: [(a, b) for a, b in edges(g) if a >= io and b >= io]
    a, b = hidden_edges(0)[0]
    assert (b, a) not in edges(0)
    add_conn(0, b, a)                                          # two-node cycle
    r = int(np.flatnonzero(pop.conn_in[1] >= 0)[0])
    add_conn(1, int(pop.conn_in[1, r]), int(pop.conn_out[1, r]), en=0)   # duplicate marking
    add_conn(2, 10 ** 6, int(pop.node_key[2][pop.node_key[2] >= io][0]))  # dangling
    add_conn(3, int(pop.node_key[3][pop.node_key[3] >= io][0]), 0)         # into an input
    succ = {}
    for x, y in edges(4):
        succ.setdefault(x, []).append(y)
    a, b = hidden_edges(4)[0]
    path = [a, b]
    while path[-1] in succ and len(path) < 12:
        path.append(succ[path[-1]][0])
    add_conn(4, path[-1], a)                                   # closes a path of len(path)
    assert len(path) >= 4
    h = int(np.flatnonzero(pop.node_key[5] >= io)[0])
    e = int(np.flatnonzero(pop.node_key[5] < 0)[0])
    for k in ("key", "bias", "resp", "act", "agg"):            # duplicate node key
        getattr(pop, "node_" + k)[5, e] = getattr(pop, "node_" + k)[5, h]
    return pop


def test_large_genomes_defects_padded_and_ragged():
    """Defects in genomes of 500+ rows, where a workgroup of eight wavefronts
    takes a genome and, padded, its Kahn rounds run from the ready bitmap
    (more rows than threads): statuses equal the oracle's, and the valid
    genomes' fields are bit-exact; the same genomes in the ragged layout."""
    pop = _large_defective(np.random.default_rng(3))
    assert pop.N_max > 512
    want = oracle.transform_arrays(pop)["status"]
    assert sorted(set(int(x) for x in want[:6])) == sorted({oracle.CYCLE, oracle.DUP_CONN,
                                                           oracle.DANGLING, oracle.INPUT_DST,
                                                           oracle.DUP_NODE})
    assert (np.array(want[6:]) == 0).all()
    got = run_transform(pop)
    assert compare(pop, got) == pop.P - 6
    for g in range(6, pop.P):
        _check_rows(pop, got, g)
    rag = synth.to_ragged(pop)
    got = run_transform(rag)
    assert compare(rag, got) == rag.P - 6


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


def test_size_classes_ordered_on_callers_stream():
    """A ragged population of at least 2048 genomes is transformed by size
    class on side streams forked from and joined back to the caller's stream.
    On a non-default stream, copies of every output queued right after the
    call, and a second call into the same arrays queued after the copies, see
    the finished results: bitwise equal to a synchronised run's (both start
    from the same sentinel, so unwritten padding compares equal too)."""
    import torch
    import paper_2504_08339_amd as tn
    pop = synth.batching_population(P=2200)
    assert int(np.diff(pop.node_off).max()) > 400   # the population spans every class
    dp = to_device(pop)

    def fresh():
        tr = tn.Transformed(dp)
        for k in FIELDS:
            getattr(tr, k).view(torch.int32).fill_(-7)
        return tr

    ref = fresh()
    tn.transform(dp, ref)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        tr = fresh()
        tn.transform(dp, tr)
        copies = {k: getattr(tr, k).clone() for k in FIELDS}
        tn.transform(dp, tr)
        again = {k: getattr(tr, k).clone() for k in FIELDS}
    s.synchronize()
    for k in FIELDS:
        assert torch.equal(copies[k].view(torch.int32), getattr(ref, k).view(torch.int32)), k
        assert torch.equal(again[k].view(torch.int32), getattr(ref, k).view(torch.int32)), k


def test_size_classes_under_graph_capture():
    """Captured into a graph, the size classes of a large ragged population are
    launched one after another on the capturing stream. Three replays, each
    after an eager sentinel fill and a synchronisation, each equal the eager
    call bit for bit."""
    import torch
    import paper_2504_08339_amd as tn
    pop = synth.batching_population(P=2100)
    dp = to_device(pop)
    ref = tn.Transformed(dp)
    for k in FIELDS:
        getattr(ref, k).view(torch.int32).fill_(-7)
    tn.transform(dp, ref)
    torch.cuda.synchronize()
    tr = tn.Transformed(dp)
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        tn.transform(dp, tr)          # eager warm-up on the side stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        tn.transform(dp, tr)
    for rep in range(3):
        for k in FIELDS:
            getattr(tr, k).view(torch.int32).fill_(-7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for k in FIELDS:
            assert torch.equal(getattr(tr, k).view(torch.int32),
                               getattr(ref, k).view(torch.int32)), (rep, k)


def test_deterministic_reruns():
    pop = synth.batching_population(P=300)
    a = run_transform(pop)
    b = run_transform(pop)
    for k in a:
        assert np.array_equal(a[k], b[k]), k


def _check_rows(pop, got, g):
    """Replays the level-by-level evaluation with the assigned value rows and
    checks that no row is overwritten while a later level still reads it."""
    ns, rb, cs = blocks(pop, g)
    n = int(got["n_valid"][g])
    order = got["order"][ns][:n]
    level = got["level"][ns][:n]
    row = got["pos_row"][ns][:n]
    rp = got["row_ptr"][rb:rb + n + 1]
    es = got["edge_src"][cs]
    keys = pop.node_rows(g)["key"][order]
    is_in = keys < pop.n_in
    is_out = (keys >= pop.n_in) & (keys < pop.n_in + pop.n_out)
    last_lvl = np.full(n, -1)
    for p in range(n):
        for e in range(rp[p], rp[p + 1]):
            last_lvl[es[e]] = max(last_lvl[es[e]], level[p])
    assert len(set(row[is_in].tolist())) == int(is_in.sum())
    holder = {}                                   # row -> position currently holding it
    for p in np.flatnonzero(is_in):
        holder[row[p]] = p
    for L in range(int(level.max()) + 1 if n else 0):
        written = [p for p in range(n) if level[p] == L and not is_in[p]]
        assert len({row[p] for p in written}) == len(written)
        for p in written:
            q = holder.get(row[p])
            if q is not None:   # the previous holder must be dead before level L
                assert not is_out[q]
                assert last_lvl[q] < L, (g, p, q)
            holder[row[p]] = p
    for p in np.flatnonzero(is_out):
        assert holder[row[p]] == p                # outputs survive to the end
    assert int(got["n_rows"][g]) == (int(row.max()) + 1 if n else 0) <= n


@pytest.mark.parametrize("name", ["control", "batching", "cppn"])
def test_value_rows_reuse_is_safe(name):
    pop = {"control": lambda: synth.control_population(P=300),
           "batching": lambda: synth.batching_population(P=300),
           "cppn": lambda: synth.cppn_population(P=300)}[name]()
    got = run_transform(pop)
    for g in range(pop.P):
        _check_rows(pop, got, g)
    rows = got["n_rows"][:pop.P]
    nv = got["n_valid"][:pop.P]
    assert (rows < nv).mean() > 0.5           # reuse actually saves rows


def _check_prog(pop, got, g):
    """The packed program of genome g: its fields mirror the position arrays,
    and replaying it one position after the other never reads a row that was
    overwritten; its row count is the largest number of values live at once."""
    ns, rb, cs = blocks(pop, g)
    n = int(got["n_valid"][g])
    rp = got["row_ptr"][rb:rb + n + 1]
    es = got["edge_src"][cs]
    pn = got["prog_node"].reshape(-1, 4)[ns][:n]
    pe = got["prog_edge"].reshape(-1, 2)[cs][:rp[n] if n else 0]
    keys = pop.node_rows(g)["key"][got["order"][ns][:n]]
    n_in, nio = pop.n_in, pop.n_in + pop.n_out
    assert np.array_equal(pn[:, 0], rp[1:])
    assert np.array_equal(pn[:, 2], got["pos_bias"][ns][:n].view(np.int32))
    assert np.array_equal(pn[:, 3], got["pos_resp"][ns][:n].view(np.int32))
    fn = got["pos_fn"][ns][:n]
    inp = keys < n_in
    assert np.array_equal(pn[inp, 1], fn[inp])
    assert np.array_equal(pn[~inp, 1] & 0xffff, fn[~inp] & 0xffff)
    prow = np.where(inp, keys, (pn[:, 1] >> 16) & 0x7fff)
    assert np.array_equal(pe[:, 0], prow[es[:len(pe)]])
    assert np.array_equal(pe[:, 1], got["edge_w"][cs][:len(pe)].view(np.int32))
    last = np.full(n, -1)
    for p in range(n):
        for e in range(rp[p], rp[p + 1]):
            last[es[e]] = max(last[es[e]], p)
    holder = {int(k): p for p, k in enumerate(keys) if k < n_in}
    live_max = n_in
    for p in range(n):
        if inp[p]:
            continue
        for e in range(rp[p], rp[p + 1]):
            assert holder[int(pe[e, 0])] == es[e], (g, p, e)   # source still in its row
        r = int(prow[p])
        q = holder.get(r)
        if q is not None:   # the row's previous value is dead from p on
            assert not (n_in <= keys[q] < nio)
            assert last[q] <= p, (g, p, q)
        holder[r] = p
        live = sum(1 for s in range(n) if (inp[s] and last[s] > p) or (
            not inp[s] and s < p and ((n_in <= keys[s] < nio) or last[s] > p))) + 1
        live_max = max(live_max, live)
    for p in np.flatnonzero((keys >= n_in) & (keys < nio)):
        assert holder[int(prow[p])] == p
    assert int(got["prog_rows"][g]) == live_max
    assert prow.max(initial=0) < live_max
    # the same program as 16-word records of the non-input positions
    rec = got["prog_rec"].reshape(-1, 16)[ns]
    nr = pop.node_rows(g)
    order = got["order"][ns][:n]
    zrow = int(got["prog_rows"][g])
    r = 0
    for p in range(n):
        if inp[p]:
            continue
        w = rec[r]
        e0, ne = int(rp[p]), int(rp[p + 1] - rp[p])
        act, agg = int(nr["act"][order[p]]), int(nr["agg"][order[p]])
        assert w[0] == act | (agg << 3) | (int(prow[p]) << 6) | (ne << 17), (g, p)
        assert w[1] == got["pos_bias"][ns][p:p + 1].view(np.int32)[0]
        assert w[2] == got["pos_resp"][ns][p:p + 1].view(np.int32)[0]
        assert w[3] == e0 + 6
        for i in range(6):
            if i < ne:
                assert (w[4 + 2 * i], w[5 + 2 * i]) == (pe[e0 + i, 0], pe[e0 + i, 1])
            else:
                assert (w[4 + 2 * i], w[5 + 2 * i]) == (zrow, 0)
        r += 1
    assert np.all(rec[r:] == 0)


@pytest.mark.parametrize("name", ["control", "batching", "cppn"])
def test_packed_program_rows(name):
    pop = {"control": lambda: synth.control_population(P=200),
           "batching": lambda: synth.batching_population(P=120),
           "cppn": lambda: synth.cppn_population(P=200)}[name]()
    got = run_transform(pop)
    for g in range(pop.P):
        if got["status"][g]:
            assert got["prog_rows"][g] == 0
            continue
        _check_prog(pop, got, g)
    # the program needs no more rows than the level-parallel assignment
    ok = got["status"][:pop.P] == 0
    assert np.all(got["prog_rows"][:pop.P][ok] <= got["n_rows"][:pop.P][ok])


def test_packed_program_malformed_and_holed():
    rng = np.random.default_rng(4)
    for pop in (_malformed(), synth.insert_holes(synth.control_population(P=60), rng),
                synth.permute_rows(synth.control_population(P=60), rng)):
        got = run_transform(pop)
        for g in range(pop.P):
            if got["status"][g] == 0:
                _check_prog(pop, got, g)
