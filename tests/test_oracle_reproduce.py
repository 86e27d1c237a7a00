"""Pins of the oracle's crossover and mutation (TensorNEAT Section 3.2).

Each pin checks the oracle against something other than its own code: set
algebra over keys and markings, the forward oracle (a split with weight 1 in
and the old weight out around an identity node of bias 0 leaves the network's
outputs unchanged), the transform oracle's cycle and dangling flags, brute
force over every (source, destination) pick of small genomes, and hand-worked
attribute updates. A last group plants mistakes and checks they are caught.
"""
import dataclasses

import numpy as np
import pytest

import oracle
import oracle.reproduce as orp
import synth
from helpers import load_golden, population_from_rows

P_DEF = orp.MutationParams()
GOLD = load_golden("reproduction.json")


def _draws(pop, n, seed):
    return synth.reproduction_draws(n, orp.n_uniform(pop.N_max, pop.C_max),
                                    orp.n_normal(pop.N_max, pop.C_max), seed)


def _genes(rows):
    nodes = {int(rows.key[r]): (rows.bias[r], rows.resp[r], rows.act[r], rows.agg[r])
             for r in rows.valid_nodes()}
    conns = {(int(rows.cin[r]), int(rows.cout[r])): (rows.w[r], rows.en[r])
             for r in rows.valid_conns()}
    return nodes, conns


def _as_pop(pop, arrays):
    return synth.Population(pop.n_in, pop.n_out, pop.N_max, pop.C_max,
                            *[arrays[k] for k in ("node_key", "node_bias", "node_resp",
                                                  "node_act", "node_agg", "conn_in",
                                                  "conn_out", "conn_w", "conn_en")])


def _rows_equal(a, b):
    return all(np.array_equal(getattr(a, f.name), getattr(b, f.name))
               for f in dataclasses.fields(a))


# ---- crossover ---------------------------------------------------------------

def test_crossover_of_identical_parents_is_the_parent():
    pop = synth.control_population(P=20)
    U, _ = _draws(pop, 20, 1)
    for g in range(pop.P):
        p = orp.Rows.of(pop, g)
        assert _rows_equal(orp.crossover(p, orp.Rows.of(pop, g), U[g]), p)


@pytest.mark.parametrize("coin", [0.9, 0.1, None])
def test_crossover_by_set_algebra(coin):
    pop = synth.control_population(P=30)
    U, _ = _draws(pop, 15, 2)
    for c in range(15):
        a, b = orp.Rows.of(pop, 2 * c), orp.Rows.of(pop, 2 * c + 1)
        u = U[c].copy()
        if coin is not None:
            u[:] = coin
        child = orp.crossover(a, b, u)
        na, ca = _genes(a)
        nb, cb = _genes(b)
        nc, cc = _genes(child)
        # the child holds exactly the fitter parent's genes, in its rows
        assert set(nc) == set(na) and set(cc) == set(ca)
        assert np.array_equal(child.key, a.key) and np.array_equal(child.cin, a.cin)
        for k in na:
            r = int(np.flatnonzero(a.key == k)[0])
            take_b = k in nb and u[orp.N_STRUCT + r] < 0.5
            assert nc[k] == (nb[k] if take_b else na[k])
        for m in ca:
            r = [q for q in a.valid_conns() if (a.cin[q], a.cout[q]) == m][0]
            take_b = m in cb and u[orp.N_STRUCT + pop.N_max + r] < 0.5
            assert cc[m] == (cb[m] if take_b else ca[m])
        if coin == 0.9:
            assert _rows_equal(child, a)


# ---- structural mutations ------------------------------------------------------

def _only(**kw):
    base = dict(node_add=0.0, conn_add=0.0, bias_mutate_rate=0.0, bias_replace_rate=0.0,
                weight_mutate_rate=0.0, weight_replace_rate=0.0)
    base.update(kw)
    return dataclasses.replace(P_DEF, **base)


def test_split_preserves_function_and_keys():
    """Add node with an identity node of bias 0 and response 1: outputs equal
    the parent's (float64, up to the sum order of the moved term)."""
    pop = synth.control_population(P=40)
    prm = _only(node_add=1.0, act_default=0, bias_init_std=0.0, resp_init_std=0.0)
    U, Z = _draws(pop, pop.P, 3)
    parents = np.stack([np.arange(pop.P), np.arange(pop.P)], 1)
    kids, nxt = orp.reproduce(pop, parents, U, Z, prm, next_key=10 ** 6)
    child = _as_pop(pop, kids)
    X = synth.normal_obs(pop.P, 16, pop.n_in, 4)
    Y0 = oracle.forward_population(pop, X)
    Y1 = oracle.forward_population(child, X)
    np.testing.assert_allclose(Y1, Y0, rtol=1e-12, atol=1e-12)
    splits = 0
    for g in range(pop.P):
        p, c = orp.Rows.of(pop, g), orp.Rows.of(child, g)
        pn, pc = _genes(p)
        cn, cc = _genes(c)
        new = set(cn) - set(pn)
        assert set(pn) <= set(cn) and len(new) <= 1
        if not new:
            continue
        splits += 1
        (h,) = new
        assert h >= 10 ** 6
        # first empty rows took the new node and connections
        assert int(np.flatnonzero(p.key < 0)[0]) == int(np.flatnonzero(c.key == h)[0])
        (a, b), = [m for m in pc if pc[m][1] and not cc[m][1]]
        assert cc[(a, h)] == (np.float32(1.0), 1) and cc[(h, b)] == (pc[(a, b)][0], 1)
        free = [r for r in range(pop.C_max) if p.cin[r] < 0]
        assert (c.cin[free[0]], c.cout[free[0]]) == (a, h)
        assert (c.cin[free[1]], c.cout[free[1]]) == (h, b)
    assert splits > 30
    assert nxt > 10 ** 6


def test_innovation_table_reuses_a_split():
    """Golden: two children splitting the same connection get one key; keys
    follow the lexicographic order of the split markings."""
    keys, nxt = orp.innovation_keys([(5, 9), (0, 3), (5, 9), (0, 7), (2, 3)], 100)
    assert keys == {(0, 3): 100, (0, 7): 101, (2, 3): 102, (5, 9): 103} and nxt == 104
    pop = synth.control_population(P=4)
    prm = _only(node_add=1.0)
    U, Z = _draws(pop, 6, 5)
    U[:, 1] = U[0, 1]                      # same pick ...
    parents = np.array([[1, 1]] * 3 + [[2, 2]] * 3)   # ... in the same parent
    kids, nxt = orp.reproduce(pop, parents, U, Z, prm, next_key=500)
    new = [set(kids["node_key"][c][kids["node_key"][c] >= 0]) - set(pop.node_key[parents[c, 0]])
           for c in range(6)]
    assert new[0] == new[1] == new[2] and len(new[0]) == 1
    assert new[3] == new[4] == new[5] and new[3] != new[0]
    assert nxt == 502


def _reaches_by_transform(rows, n_in, n_out, s, d):
    """Adding s -> d closes a cycle iff the transform oracle flags CYCLE on the
    genome with every valid connection enabled plus s -> d."""
    nodes = [[int(rows.key[r]), 0.0, 1.0, 0, 0] for r in rows.valid_nodes()]
    conns = [[int(rows.cin[r]), int(rows.cout[r]), 1.0, 1] for r in rows.valid_conns()]
    conns.append([s, d, 1.0, 1])
    pop = population_from_rows([(nodes, conns)], n_in, n_out)
    return bool(oracle.transform(oracle.decode(pop, 0)).status & oracle.CYCLE)


@pytest.mark.parametrize("allow_cycles", [False, True])
def test_add_connection_brute_force(allow_cycles):
    """Every (source, destination) pick of small genomes: the connection is
    added exactly when the endpoints differ, the marking is absent and (for
    feedforward genomes) it closes no cycle."""
    pop = synth.grow_population(12, 3, 2, 16, 40, 12, np.random.default_rng(6),
                                hidden_acts=("tanh",), output_acts=("tanh",), disable_p=0.3)
    prm = dataclasses.replace(_only(conn_add=1.0), allow_cycles=allow_cycles)
    U, Z = _draws(pop, 1, 7)
    added = refused_cycle = 0
    for g in range(pop.P):
        par = orp.Rows.of(pop, g)
        srcs = [r for r in par.valid_nodes() if not (3 <= par.key[r] < 5)]
        dsts = [r for r in par.valid_nodes() if not (0 <= par.key[r] < 3)]
        _, pc = _genes(par)
        for i in range(len(srcs)):
            for j in range(len(dsts)):
                u = U[0].copy()
                u[5] = (i + 0.5) / len(srcs)
                u[6] = (j + 0.5) / len(dsts)
                child = orp.mutate(orp.Rows.of(pop, g), u, Z[0], prm, 3, 2, None, None)
                s, d = int(par.key[srcs[i]]), int(par.key[dsts[j]])
                _, cc = _genes(child)
                cyc = _reaches_by_transform(par, 3, 2, s, d)
                want = s != d and (s, d) not in pc and (allow_cycles or not cyc)
                assert ((s, d) in cc and (s, d) not in pc) == want, (g, s, d)
                if want:
                    added += 1
                    r = int(np.flatnonzero(par.cin < 0)[0])
                    assert (child.cin[r], child.cout[r], child.en[r]) == (s, d, 1)
                refused_cycle += cyc and s != d and (s, d) not in pc
    assert added > 60 and refused_cycle > 10, (added, refused_cycle)


def test_delete_node_leaves_no_dangling_connection():
    pop = synth.control_population(P=60)
    prm = _only(node_delete=1.0)
    U, Z = _draws(pop, pop.P, 8)
    kids, _ = orp.reproduce(pop, np.stack([np.arange(60), np.arange(60)], 1), U, Z, prm, 10 ** 5)
    child = _as_pop(pop, kids)
    removed = 0
    for g in range(pop.P):
        st = oracle.transform(oracle.decode(child, g)).status
        assert st == 0, (g, st)
        pn, _ = _genes(orp.Rows.of(pop, g))
        cn, cc = _genes(orp.Rows.of(child, g))
        gone = set(pn) - set(cn)
        assert len(gone) <= 1 and all(k >= pop.n_in + pop.n_out for k in gone)
        assert not any(k in m for m in cc for k in gone)
        removed += len(gone)
    assert removed > 40


def test_delete_connection_empties_one_row():
    pop = synth.control_population(P=20)
    prm = _only(conn_delete=1.0)
    U, Z = _draws(pop, pop.P, 9)
    kids, _ = orp.reproduce(pop, np.stack([np.arange(20), np.arange(20)], 1), U, Z, prm, 10 ** 5)
    for g in range(pop.P):
        before = int(np.count_nonzero(pop.conn_in[g] >= 0))
        after = int(np.count_nonzero(kids["conn_in"][g] >= 0))
        assert after == before - 1


def test_no_room_no_change():
    """A genome whose node rows are all taken cannot be split."""
    pop = synth.xor_population(P=10)
    full = synth.subset(pop, range(10))
    rows = full.node_key >= 0
    for g in range(full.P):
        free = np.flatnonzero(~rows[g])
        full.node_key[g, free] = 1000 + np.arange(free.size) + 100 * g
    U, Z = _draws(full, 10, 10)
    kids, nxt = orp.reproduce(full, np.stack([np.arange(10), np.arange(10)], 1), U, Z,
                              _only(node_add=1.0), 5000)
    assert nxt == 5000 and np.array_equal(kids["node_key"], full.node_key)


# ---- attributes ------------------------------------------------------------------

@pytest.mark.parametrize("case", GOLD["attribute_updates"], ids=lambda c: c["name"])
def test_attribute_rule_by_hand(case):
    got = orp._mut_float(case["v"], case["u"], case["z"], case["init_mean"], case["init_std"],
                         case["power"], case["rate"], case["replace"])
    assert got == np.float32(case["expected"])


def test_attribute_mutation_rates_and_elites():
    pop = synth.control_population(P=200)
    U, Z = _draws(pop, pop.P, 11)
    parents = np.stack([np.arange(pop.P), np.arange(pop.P)], 1)
    parents[:10, 1] = -1                                   # elites
    prm = _only(weight_mutate_rate=0.8, weight_replace_rate=0.1)
    kids, _ = orp.reproduce(pop, parents, U, Z, prm, 10 ** 5)
    for k in kids:
        assert np.array_equal(kids[k][:10], getattr(pop, k)[:10]), k   # elites copied as is
    valid = pop.conn_in[10:] >= 0
    changed = kids["conn_w"][10:][valid] != pop.conn_w[10:][valid]
    assert abs(changed.mean() - 0.9) < 0.01                 # mutated or replaced
    assert np.array_equal(kids["conn_in"], pop.conn_in)     # no structure change


def test_activation_replacement_uses_the_options():
    pop = synth.control_population(P=50)
    U, Z = _draws(pop, pop.P, 12)
    prm = _only(act_replace_rate=1.0, act_options=(4, 1, 6))
    kids, _ = orp.reproduce(pop, np.stack([np.arange(50), np.arange(50)], 1), U, Z, prm, 10 ** 5)
    hid = (pop.node_key >= pop.n_in)
    vals = kids["node_act"][hid]
    assert set(np.unique(vals)) == {1, 4, 6}
    assert np.array_equal(kids["node_act"][pop.node_key < pop.n_in],
                          pop.node_act[pop.node_key < pop.n_in])


# ---- planted mistakes ---------------------------------------------------------------

def _fails(fn, *a):
    try:
        fn(*a)
    except AssertionError:
        return True
    return False


def test_planted_swapped_split_weights(monkeypatch):
    orig = orp.mutate

    def wrong(child, U, Z, prm, n_in, n_out, split_row, split_key):
        if split_row is not None:
            w = child.w[split_row]
            out = orig(child, U, Z, prm, n_in, n_out, split_row, split_key)
            r = [q for q in out.valid_conns() if out.cin[q] == split_key][0]
            s = [q for q in out.valid_conns() if out.cout[q] == split_key][0]
            out.w[r], out.w[s] = np.float32(1.0), w
            return out
        return orig(child, U, Z, prm, n_in, n_out, split_row, split_key)
    monkeypatch.setattr(orp, "mutate", wrong)
    assert _fails(test_split_preserves_function_and_keys)


def test_planted_missing_cycle_check(monkeypatch):
    monkeypatch.setattr(orp, "_reaches", lambda *a: False)
    assert _fails(test_add_connection_brute_force, False)


def test_planted_crossover_coin_inverted(monkeypatch):
    orig = orp.crossover
    monkeypatch.setattr(orp, "crossover", lambda a, b, U: orig(a, b, 1.0 - U))
    assert _fails(test_crossover_by_set_algebra, None)
