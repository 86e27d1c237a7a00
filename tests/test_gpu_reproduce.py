"""GPU parity of tn_reproduce (tensorized crossover and mutation, Section 3.2)
against the oracle: given the same parents and draws, every row of every
child and the next free key must be equal bit for bit (the integer decisions
are taken in float32 on both sides, and each float update is the same two
float32 roundings)."""
import dataclasses

import numpy as np
import pytest
import torch

import oracle.reproduce as orp
import synth
from gpu_util import FIELDS, host, tensor, to_device
from helpers import population_from_rows

pytestmark = pytest.mark.gpu

BUSY = dict(node_add=0.5, node_delete=0.3, conn_add=0.7, conn_delete=0.3,
            act_replace_rate=0.3, agg_replace_rate=0.2, act_options=(3, 0, 2, 1),
            agg_options=(4, 0), resp_mutate_rate=0.3, resp_mutate_power=0.2,
            resp_replace_rate=0.2, resp_init_std=0.5)


def _gpu(pop, parents, U, Z, prm, next_key):
    import paper_2504_08339_amd as tn
    kids, nk = tn.reproduce(to_device(pop), tensor(parents.astype(np.int32)), tensor(U),
                            tensor(Z), tn.MutationParams(**dataclasses.asdict(prm)), next_key)
    return {k: host(kids.t[k]) for k in FIELDS}, int(host(nk)[0])


def _check(pop, parents, seed, prm=None, next_key=None):
    prm = prm or orp.MutationParams()
    n = parents.shape[0]
    U, Z = synth.reproduction_draws(n, orp.n_uniform(pop.N_max, pop.C_max),
                                    orp.n_normal(pop.N_max, pop.C_max), seed)
    if next_key is None:
        next_key = int(max(pop.node_key.max(), pop.conn_in.max(), pop.conn_out.max())) + 1
    ref, ref_next = orp.reproduce(pop, parents, U, Z, prm, next_key)
    got, got_next = _gpu(pop, parents, U, Z, prm, next_key)
    for k in FIELDS:
        a, b = got[k], ref[k]
        if a.dtype == np.float32:
            a, b = a.view(np.uint32), b.astype(np.float32).view(np.uint32)
        bad = np.argwhere(a != b)
        assert bad.size == 0, f"{k}: {len(bad)} rows differ, first child/row {bad[:4].tolist()}"
    assert got_next == ref_next
    return ref, ref_next


def _parents(P, n, rng, elite_frac=0.1):
    par = rng.integers(0, P, size=(n, 2))
    par[rng.random(n) < elite_frac, 1] = -1
    return par


def test_xor_default_params_many_children():
    """XOR capacities (16 nodes / 32 connections), Appendix C defaults; 400
    children from 150 parents, so splits of one marking recur (one key)."""
    pop = synth.xor_population()
    rng = np.random.default_rng(1)
    _, nxt = _check(pop, _parents(pop.P, 400, rng), seed=11)
    assert nxt > 0


def test_control_busy_params():
    """Every structural mutation and attribute rule with high rates."""
    pop = synth.control_population(P=80)
    rng = np.random.default_rng(2)
    _check(pop, _parents(pop.P, 200, rng), seed=12, prm=orp.MutationParams(**BUSY))


def test_control_full_population():
    """1000 children of the 1000-genome control population (64 / 256 rows)."""
    pop = synth.control_population()
    rng = np.random.default_rng(3)
    _check(pop, _parents(pop.P, 1000, rng), seed=13, prm=orp.MutationParams(**BUSY))


def test_full_rows_and_capacity_limits():
    """Genomes whose node or connection rows are all taken: the additions that
    need a free row are skipped on both sides."""
    io = [[0, 0, 1, 0, 0], [1, 0, 1, 0, 0], [2, 0.5, 1, 2, 0]]
    genomes = [
        (io + [[5, 0.1, 1, 2, 0]], [[0, 5, 1.0, 1], [5, 2, 2.0, 1], [1, 2, 3.0, 1]]),  # all full
        (io + [None], [[0, 2, 1.0, 1], None, [1, 2, -1.0, 1]]),                      # one free conn
        (io + [[6, 0, 1, 2, 0]], [[0, 6, 1.0, 1], [6, 2, 1.0, 1], None]),            # no free node
        (io + [None], [None, None, None]),                                            # nothing
    ]
    pop = population_from_rows(genomes, 2, 1, N_max=4, C_max=3)
    rng = np.random.default_rng(4)
    prm = orp.MutationParams(node_add=0.9, conn_add=0.9, node_delete=0.0, conn_delete=0.0)
    for seed in range(5):
        _check(pop, _parents(pop.P, 64, rng, 0.0), seed=20 + seed, prm=prm)


def test_cycles_allowed_and_dangling_paths():
    """allow_cycles on, and reachability through keys no node row holds."""
    io = [[0, 0, 1, 0, 0], [1, 0, 1, 0, 0], [2, 0.5, 1, 2, 0]]
    genomes = [
        # 2 -> 9 -> 5 through key 9 (no node row): adding 5 -> ... must see 5 reaches 2's successors
        (io + [[5, 0, 1, 2, 0], [7, 0, 1, 2, 0]],
         [[0, 5, 1.0, 1], [5, 9, 1.0, 1], [9, 7, 1.0, 1], [7, 2, 1.0, 0], None, None]),
        (io + [[5, 0, 1, 2, 0], [7, 0, 1, 2, 0]],
         [[0, 5, 1.0, 1], [5, 7, 1.0, 1], [7, 2, 1.0, 1], None, None, None]),
    ]
    pop = population_from_rows(genomes, 2, 1, N_max=6, C_max=6)
    rng = np.random.default_rng(5)
    for allow in (False, True):
        prm = orp.MutationParams(node_add=0.0, conn_add=1.0, allow_cycles=allow)
        for seed in range(6):
            _check(pop, _parents(pop.P, 128, rng, 0.0), seed=30 + seed, prm=prm)


def test_batching_shapes_padded():
    """Large capacities (the batching population padded to 544 nodes / 2000
    connections) on a subset: several 256-row chunks per block scan."""
    pop = synth.to_padded(synth.batching_population(P=40))
    rng = np.random.default_rng(6)
    _check(pop, _parents(pop.P, 48, rng), seed=40, prm=orp.MutationParams(**BUSY))


def test_degenerate_calls():
    import paper_2504_08339_amd as tn
    pop = synth.xor_population(P=8)
    dp = to_device(pop)
    nu, nz = tn.reproduce_draws(pop.N_max, pop.C_max)
    assert (nu, nz) == (orp.n_uniform(pop.N_max, pop.C_max), orp.n_normal(pop.N_max, pop.C_max))
    # no children: the next free key is the one given
    empty = torch.zeros((0, 2), dtype=torch.int32, device="cuda")
    kids, nk = tn.reproduce(dp, empty, torch.zeros((0, nu), device="cuda"),
                            torch.zeros((0, nz), device="cuda"), None, 77)
    assert int(host(nk)[0]) == 77 and kids.P == 0
    # a first parent outside [0, P): an all-empty child; a second one: an elite
    par = tensor(np.array([[-3, 1], [8, 0], [2, 8], [2, -1]], np.int32))
    U, Z = synth.reproduction_draws(4, nu, nz, 1)
    kids, nk = tn.reproduce(dp, par, tensor(U), tensor(Z), None, 100)
    got = {k: host(kids.t[k]) for k in FIELDS}
    for c in (0, 1):
        assert (got["node_key"][c] == -1).all() and (got["conn_in"][c] == -1).all()
        assert (got["conn_w"][c] == 0).all() and (got["node_bias"][c] == 0).all()
    for c in (2, 3):
        for k in FIELDS:
            assert np.array_equal(got[k][c], getattr(pop, k)[2]), k
    assert int(host(nk)[0]) == 100


def test_bad_params_rejected_before_launch():
    import paper_2504_08339_amd as tn
    pop = synth.xor_population(P=4)
    dp = to_device(pop)
    nu, nz = tn.reproduce_draws(pop.N_max, pop.C_max)
    par = tensor(np.array([[0, 1]], np.int32))
    U, Z = synth.reproduction_draws(1, nu, nz, 1)
    for bad in (dict(node_add=1.5), dict(conn_delete=-0.1), dict(act_options=()),
                dict(agg_options=tuple(range(9))), dict(act_default=300)):
        with pytest.raises((tn.TNError, ValueError)):
            tn.reproduce(dp, par, tensor(U), tensor(Z), tn.MutationParams(**bad), 10)
