"""Pins of the oracle's NEAT generation (Algorithm 1's loop body; readings in
oracle/neat.py): hand-worked speciation on genomes that differ in one weight
(the distance is then c_h |dw| / n, a line), hand-worked offspring counts and
stagnation, parent selection rules, the float32 distance against the pinned
float64 one, the initial population against hand-built rows and the forward
oracle, whole-generation invariants, and planted mistakes."""
import dataclasses
import math

import numpy as np
import pytest

import oracle
import oracle.neat as on
import oracle.reproduce as orp
import synth
from helpers import population_from_rows

IO = [[0, 0.0, 1.0, 0, 0], [1, 0.0, 1.0, 0, 0], [2, 0.0, 1.0, 1, 0]]


def _line_pop(ws, extra=None):
    """Genomes 2 -> 1 with one hidden node 5 whose in-weight is w_g: every
    pair shares its genes, so delta = 0.5 * |w_g - w_h| / 3 (3 connections)."""
    genomes = []
    for w in ws:
        genomes.append((IO + [[5, 0.0, 1.0, 2, 0]],
                        [[0, 5, float(w), 1], [5, 2, 1.0, 1], [1, 2, 1.0, 1]]))
    return population_from_rows(genomes, 2, 1, N_max=6, C_max=6)


def test_distance_f32_matches_float64_distance():
    pop = synth.control_population(P=40)
    genes = [on._genes_of_rows(orp.Rows.of(pop, g), pop.n_in) for g in range(pop.P)]
    for i in range(pop.P):
        for j in range(pop.P):
            d32 = on.distance_f32(genes[i], genes[j], 1.0, 0.5)
            d64, _, _ = oracle.distance_nodes(oracle.node_genes(pop, i), oracle.node_genes(pop, j),
                                              1.0, 0.5)
            assert abs(float(d32) - d64) <= (1e-5 + 300 * 2.0 ** -24) * abs(d64) + 1e-7


def test_distance_f32_on_the_line():
    pop = _line_pop([0.0, 0.75, 3.0])
    g = [on._genes_of_rows(orp.Rows.of(pop, i), 2) for i in range(3)]
    assert on.distance_f32(g[0], g[1], 1.0, 0.5) == np.float32(0.5 * 0.75 / 3)
    assert on.distance_f32(g[0], g[2], 1.0, 0.5) == np.float32(0.5)
    assert on.distance_f32(g[2], g[2], 1.0, 0.5) == 0


def test_speciation_by_hand():
    """Weights 0, 10, 0.5, 20, 10.4, 100, 0.2 with threshold 1 (|dw| < 6) and
    at most 3 species: 0 founds slot 0, 10 slot 1, 0.5 joins 0, 20 founds slot
    2, 10.4 joins 1, then the table is full: 100 joins the nearest (20, slot
    2) and 0.2 joins slot 0."""
    pop = _line_pop([0.0, 10.0, 0.5, 20.0, 10.4, 100.0, 0.2])
    prm = on.NeatParams(compatibility_threshold=1.0, max_species=3)
    sp, founded = on.speciate(pop, on.SpeciesTable.empty(3), prm)
    assert list(sp) == [0, 1, 0, 2, 1, 2, 0] and founded == [0, 1, 2]


def test_speciation_against_existing_representatives():
    """Slots 1 and 3 alive with representatives at weights 0 and 0 (a tie):
    genomes near 0 join slot 1 (lowest); far ones found slots 0, 2."""
    reps = _line_pop([0.0, 0.0])
    table = on.SpeciesTable.empty(4)
    for s, g in ((1, 0), (3, 1)):
        table.alive[s] = True
        table.reps[s] = orp.Rows.of(reps, g)
    pop = _line_pop([1.0, 50.0, -3.0, 51.0, 200.0])
    prm = on.NeatParams(compatibility_threshold=1.0, max_species=4)
    sp, founded = on.speciate(pop, table, prm)
    # 1 and -3 within 6 of 0 -> slot 1; 50 founds 0; 51 joins 0; 200 founds 2
    assert list(sp) == [1, 0, 1, 0, 2] and founded == [0, 2]


def test_allocation_by_hand():
    """Two species of five (fitness 4 and 2), sizes 5 and 5: af = 1 and 0,
    targets 10 and 0, spawn 7.5 and 2.5 with change rate 1/2, shares 7.5 and
    2.5, floors 7 and 2, the last child to the tie's lower slot: 8 and 2."""
    sp = np.array([0] * 5 + [1] * 5)
    fit = np.array([4.0] * 5 + [2.0] * 5, np.float32)
    table = on.SpeciesTable.empty(3)
    table.alive[:2] = True
    table.size[:2] = 5
    table.best[:2] = -np.inf
    counts, surv, best, last = on.allocate(fit, sp, table, [], 7, on.NeatParams(), 10)
    assert list(counts) == [8, 2, 0] and list(surv) == [True, True, False]
    assert list(best[:2]) == [4.0, 2.0] and list(last[:2]) == [7, 7]


def test_stagnation_by_hand():
    """Slots 0, 1, 2 (members' fitness [3, 0], [2, 2], [1.5, 0.5]) with last
    improvements at generations 0, 0, 10 and bests above their current
    fitness; at generation 20 with max_stagnation 15 and species_elitism 1:
    slot 0 (species fitness 3, the largest member) is protected, slot 1
    (stagnant 20 generations) is dropped, slot 2 (10) survives."""
    sp = np.array([0, 0, 1, 1, 2, 2])
    fit = np.array([3.0, 0.0, 2.0, 2.0, 1.5, 0.5], np.float32)
    table = on.SpeciesTable.empty(3)
    table.alive[:] = True
    table.best[:] = 9.0
    table.last[:] = [0, 0, 10]
    table.size[:] = 2
    prm = on.NeatParams(species_elitism=1, max_stagnation=15)
    counts, surv, best, last = on.allocate(fit, sp, table, [], 20, prm, 6)
    assert list(surv) == [True, False, True] and counts[1] == 0 and counts.sum() == 6


def test_parent_selection_rules():
    rng = np.random.default_rng(3)
    P = 40
    fit = rng.integers(0, 5, size=P).astype(np.float32)     # many ties
    sp = rng.integers(0, 3, size=P)
    rank, order = on.rank_members(fit, sp)
    counts = np.array([15, 0, 25])
    sel = rng.random((P, 2), dtype=np.float32)
    prm = on.NeatParams(genome_elitism=2, survival_threshold=0.2)
    par = on.select_parents(fit, order, counts, sel, prm)
    assert par.shape == (P, 2)
    c = 0
    for s in (0, 2):
        ms = order[s]
        k = max(1, math.ceil(0.2 * len(ms)))
        for i in range(counts[s]):
            a, b = par[c]
            if i < min(2, len(ms)):
                assert (a, b) == (ms[i], -1)
            else:
                assert a in ms[:k] and b in ms[:k]
                assert fit[a] > fit[b] or (fit[a] == fit[b] and a <= b)
            c += 1
    # ranks: largest fitness first, ties by lower index
    for s, ms in order.items():
        for x, y in zip(ms, ms[1:]):
            assert fit[x] > fit[y] or (fit[x] == fit[y] and x < y)


def test_initial_population():
    prm = orp.MutationParams(act_default=1)
    N, C = 8, 8
    Z = synth.reproduction_draws(3, 1, orp.n_normal(N, C), 4)[1]
    arr = on.init_population(3, 3, 2, N, C, Z, prm)
    assert list(arr["node_key"][0]) == [0, 1, 2, 3, 4, -1, -1, -1]
    assert list(arr["conn_in"][1]) == [0, 0, 1, 1, 2, 2, -1, -1]
    assert list(arr["conn_out"][1]) == [3, 4, 3, 4, 3, 4, -1, -1]
    assert np.array_equal(arr["conn_w"][2, :6], Z[2, 4 + 2 * N: 4 + 2 * N + 6])
    assert np.array_equal(arr["node_bias"][2, :5], Z[2, 4:14:2])
    assert (arr["node_resp"][:, :5] == 1).all() and (arr["node_act"][:, :5] == 1).all()
    pop = synth.Population(3, 2, N, C, *[arr[k] for k in (
        "node_key", "node_bias", "node_resp", "node_act", "node_agg", "conn_in", "conn_out",
        "conn_w", "conn_en")])
    X = np.array([[0.5, -1.0, 1.0]])
    for g in range(3):
        W = arr["conn_w"][g, :6].reshape(3, 2).astype(np.float64)
        want = 1 / (1 + np.exp(-(X @ W + arr["node_bias"][g, 3:5])))
        got = oracle.forward(oracle.decode(pop, g), oracle.transform(oracle.decode(pop, g)), X)
        assert np.allclose(got, want, rtol=1e-12)


def _xor_start(P=150, seed=1):
    mp = orp.MutationParams(act_default=1)
    prm = on.NeatParams(mutation=mp)
    N, C = 16, 32
    Z = synth.reproduction_draws(P, 1, orp.n_normal(N, C), seed)[1]
    arr = on.init_population(P, 3, 1, N, C, Z, mp)
    pop = synth.Population(3, 1, N, C, *[arr[k] for k in (
        "node_key", "node_bias", "node_resp", "node_act", "node_agg", "conn_in", "conn_out",
        "conn_w", "conn_en")])
    return pop, prm


def test_generation_invariants_over_several_generations():
    pop, prm = _xor_start()
    table = on.SpeciesTable.empty(prm.max_species)
    rng = np.random.default_rng(5)
    nk = 4
    best_prev = -np.inf
    for gen in range(6):
        X, T = synth.xor_inputs(), synth.xor_targets()
        Y = oracle.forward_population(pop, X)
        fit = np.array([oracle.xor_fitness(Y[g], T) for g in range(pop.P)], np.float32)
        sel = rng.random((pop.P, 2), dtype=np.float32)
        U, Z = synth.reproduction_draws(pop.P, orp.n_uniform(16, 32), orp.n_normal(16, 32), gen)
        kids, table, sp, par, nk = on.generation(pop, fit, table, gen, prm, sel, U, Z, nk)
        assert par.shape == (pop.P, 2) and (sp >= 0).all()
        assert table.alive.sum() <= prm.max_species
        assert fit.max() >= best_prev   # the best genome is an elite of its species
        best_prev = fit.max()
        # elites are the parents' rows unchanged
        for c in np.flatnonzero(par[:, 1] < 0):
            assert np.array_equal(kids["conn_w"][c], pop.conn_w[par[c, 0]])
        pop = synth.Population(3, 1, 16, 32, *[kids[k] for k in (
            "node_key", "node_bias", "node_resp", "node_act", "node_agg", "conn_in", "conn_out",
            "conn_w", "conn_en")])


# ---- planted mistakes --------------------------------------------------------

def test_planted_no_change_rate_is_caught(monkeypatch):
    real = on.allocate

    def no_rate(fit, sp, table, founded, gen, prm, P):
        return real(fit, sp, table, founded, gen,
                    dataclasses.replace(prm, spawn_number_change_rate=1.0), P)

    monkeypatch.setattr(on, "allocate", no_rate)
    with pytest.raises(AssertionError):
        test_allocation_by_hand()


def test_planted_distance_without_attributes_is_caught(monkeypatch):
    real = on.distance_f32
    monkeypatch.setattr(on, "distance_f32", lambda a, b, c_d, c_h: real(a, b, c_d, 0.0))
    with pytest.raises(AssertionError):
        test_speciation_by_hand()


def test_planted_mean_species_fitness_is_caught(monkeypatch):
    # the oracle's max over a species' member fitness becomes a mean (a max of
    # two arguments stays a max)
    import builtins

    def planted(*args):
        if len(args) == 1:
            return np.float32(np.mean(list(args[0])))
        return builtins.max(*args)

    monkeypatch.setattr(on, "max", planted, raising=False)
    with pytest.raises(AssertionError):
        test_stagnation_by_hand()


def test_planted_rank_ties_to_higher_index_are_caught(monkeypatch):
    real = on.rank_members

    def reversed_ties(fit, sp):
        rank, order = real(fit, sp)
        for s, ms in order.items():
            order[s] = sorted(ms, key=lambda g: (-float(fit[g]), -g))
        return rank, order

    monkeypatch.setattr(on, "rank_members", reversed_ties)
    with pytest.raises(AssertionError):
        test_parent_selection_rules()
