"""GPU parity of the NEAT generation (tn_neat_init, tn_neat_generation)
against the oracle (oracle/neat.py), bit for bit: initial rows, the species
of every genome, the parent pairs, every child row, the species table and the
next free key. Chains of generations are driven by fitness the oracle computes
from its own population (the XOR fitness of Section 5.1's benchmark, rounded
to float32), fed to both sides: every decision then has the same float32
inputs on both sides. A last test runs the whole loop on the GPU (fitness by
tn_forward_loss) and checks its invariants."""
import dataclasses

import numpy as np
import pytest
import torch

import oracle
import oracle.neat as on
import oracle.reproduce as orp
import synth
from gpu_util import FIELDS, host, tensor

pytestmark = pytest.mark.gpu
N, C = 16, 32


def _tn_params(prm: on.NeatParams):
    import paper_2504_08339_amd as tn
    d = {f.name: getattr(prm, f.name) for f in dataclasses.fields(prm) if f.name != "mutation"}
    return tn.NeatParams(mutation=tn.MutationParams(**dataclasses.asdict(prm.mutation)), **d)


def _pop_of(arrays, n_in=3, n_out=1):
    return synth.Population(n_in, n_out, N, C, *[arrays[k] for k in FIELDS])


def _bits(a):
    a = np.asarray(a)
    return a.view(np.uint32) if a.dtype == np.float32 else a


def _same(got, ref, what):
    assert np.array_equal(_bits(got), _bits(ref)), what


def _xor_fitness(pop):
    X, T = synth.xor_inputs(), synth.xor_targets()
    Y = oracle.forward_population(pop, X)
    return np.array([oracle.xor_fitness(Y[g], T) for g in range(pop.P)], np.float32)


def _start(P, prm, seed):
    import paper_2504_08339_amd as tn
    Z0 = synth.reproduction_draws(P, 1, orp.n_normal(N, C), seed)[1]
    ref = on.init_population(P, 3, 1, N, C, Z0, prm.mutation)
    dpop, table = tn.neat_init(P, 3, 1, N, C, tensor(Z0), _tn_params(prm).mutation,
                               prm.max_species)
    for k in FIELDS:
        _same(host(dpop.t[k]), ref[k], f"init {k}")
    return _pop_of(ref), dpop, table


def _chain(P, prm, generations, seed):
    import paper_2504_08339_amd as tn
    pop, dpop, dtable = _start(P, prm, seed)
    table = on.SpeciesTable.empty(prm.max_species)
    rng = np.random.default_rng(seed)
    nk = 4
    seen_species = set()
    for gen in range(generations):
        fit = _xor_fitness(pop)
        sel = rng.random((P, 2), dtype=np.float32)
        U, Z = synth.reproduction_draws(P, orp.n_uniform(N, C), orp.n_normal(N, C), 100 * seed + gen)
        kids, table, sp, par, nk_ref = on.generation(pop, fit, table, gen, prm, sel, U, Z, nk)
        dkids, dsp, dpar, dnk = tn.neat_generation(dpop, tensor(fit), gen, dtable, tensor(sel),
                                                   tensor(U), tensor(Z), nk, _tn_params(prm))
        _same(host(dsp), sp.astype(np.int32), f"gen {gen}: species")
        _same(host(dpar), par.astype(np.int32), f"gen {gen}: parents")
        for k in FIELDS:
            _same(host(dkids.t[k]), kids[k], f"gen {gen}: child {k}")
        assert int(host(dnk)[0]) == nk_ref, gen
        _same(host(dtable.alive), table.alive.astype(np.int32), f"gen {gen}: alive")
        alive = table.alive
        _same(host(dtable.best)[alive], table.best[alive], f"gen {gen}: best")
        _same(host(dtable.last_improved)[alive], table.last[alive].astype(np.int32), f"gen {gen}")
        _same(host(dtable.size), table.size.astype(np.int32), f"gen {gen}: size")
        for s in np.flatnonzero(alive):
            for k, f in zip(FIELDS, ("key", "bias", "resp", "act", "agg", "cin", "cout", "w", "en")):
                _same(host(dtable.reps[k])[s], getattr(table.reps[s], f), f"gen {gen}: rep {s} {k}")
        seen_species.update(np.unique(sp).tolist())
        pop, dpop, nk = _pop_of(kids), dkids, nk_ref
    return seen_species


def test_xor_generations_default_parameters():
    """150 genomes, Appendix C's values (sigmoid outputs), 12 generations."""
    prm = on.NeatParams(mutation=orp.MutationParams(act_default=1))
    _chain(150, prm, 12, seed=1)


def test_full_table_stagnation_and_small_threshold():
    """Three slots, a low threshold (the table fills and later genomes join
    the nearest species), stagnation after 2 generations, one protected
    species, high structural rates."""
    mut = orp.MutationParams(act_default=1, node_add=0.5, conn_add=0.8, node_delete=0.1,
                             conn_delete=0.1)
    prm = on.NeatParams(compatibility_threshold=0.6, max_species=3, max_stagnation=2,
                        species_elitism=1, genome_elitism=1, survival_threshold=0.5,
                        spawn_number_change_rate=0.8, mutation=mut)
    seen = _chain(120, prm, 10, seed=2)
    assert len(seen) == 3


def test_many_species_and_odd_sizes():
    prm = on.NeatParams(compatibility_threshold=1.2, max_species=17, genome_elitism=3,
                        mutation=orp.MutationParams(act_default=1, node_add=0.4, conn_add=0.6))
    seen = _chain(301, prm, 6, seed=3)
    assert len(seen) >= 4


def test_gpu_loop_on_xor_improves():
    """The loop with the fitness on the GPU (tn_forward_loss: 4 - SSE over the
    four XOR rows): every generation's parents are valid, the best fitness
    never falls (each species' best genome is an elite) and it rises."""
    import paper_2504_08339_amd as tn
    P = 150
    prm = _tn_params(on.NeatParams(mutation=orp.MutationParams(act_default=1)))
    g = torch.Generator(device="cuda").manual_seed(7)
    nu, nz = tn.reproduce_draws(N, C)
    pop, table = tn.neat_init(P, 3, 1, N, C, torch.randn((P, nz), device="cuda", generator=g),
                              prm.mutation, prm.max_species)
    X, T = tensor(synth.xor_inputs()), tensor(synth.xor_targets())
    nk, bests = 4, []
    for gen in range(40):
        fit, _ = tn.forward_loss(pop, tn.transform(pop), X, T, scale=-1.0, offset=4.0,
                                 store_outputs=False)
        bests.append(float(fit.max()))
        sel = torch.rand((P, 2), device="cuda", generator=g)
        U = torch.rand((P, nu), device="cuda", generator=g)
        Z = torch.randn((P, nz), device="cuda", generator=g)
        pop, sp, par, nkt = tn.neat_generation(pop, fit, gen, table, sel, U, Z, nk, prm)
        nk = int(nkt.item())
        p = host(par)
        assert (p[:, 0] >= 0).all() and (p[:, 0] < P).all() and (p[:, 1] < P).all()
        s = host(sp)
        assert (s >= 0).all() and (s < prm.max_species).all()
    assert all(b2 >= b1 for b1, b2 in zip(bests, bests[1:])), bests
    assert bests[-1] > bests[0], bests


def test_bad_parameters_rejected():
    import paper_2504_08339_amd as tn
    prm0 = on.NeatParams(mutation=orp.MutationParams(act_default=1))
    _, dpop, table = _start(8, prm0, 4)
    nu, nz = tn.reproduce_draws(N, C)
    args = (torch.zeros(8, device="cuda"), 0, table, torch.zeros((8, 2), device="cuda"),
            torch.zeros((8, nu), device="cuda"), torch.zeros((8, nz), device="cuda"), 4)
    for bad in (dict(species_elitism=0), dict(survival_threshold=0.0),
                dict(spawn_number_change_rate=1.5), dict(compatibility_threshold=float("nan"))):
        prm = _tn_params(dataclasses.replace(prm0, **bad))
        with pytest.raises(tn.TNError):
            tn.neat_generation(dpop, *args, prm)
    with pytest.raises(ValueError):
        tn.neat_generation(dpop, *args, _tn_params(dataclasses.replace(prm0, max_species=4)))
