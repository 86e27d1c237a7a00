"""GPU parity of tn_forward_recurrent (T synchronous sweeps) against the
float64 oracle, with the forward pass's tolerance: |y - y_ref| <= 1e-5 *
cond(y) + 2^-100, cond propagated through the sweeps by the oracle. Flagged
genomes give NaN and their status bits bit-exact; on acyclic sum-aggregation
genomes T sweeps past the largest level give tn_forward's bits."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import host, tensor, to_device
from helpers import load_golden, population_from_rows

pytestmark = pytest.mark.gpu
RTOL = 1e-5
ABS_FLOOR = 2.0 ** -100


def gpu_recurrent(pop, obs, T):
    import paper_2504_08339_amd as tn
    Y, st = tn.forward_recurrent(to_device(pop), tensor(obs), T, with_status=True)
    return host(Y), host(st)


def check(pop, obs, T, Y, st, genomes=None):
    idx = list(range(pop.P)) if genomes is None else list(genomes)
    ref, cond, rst = oracle.recurrent_population(pop, obs, T, genomes=idx, with_cond=True)
    return compare(Y[idx], st[idx], ref, cond, rst)


def compare(Y, st, ref, cond, rst):
    assert np.array_equal(st, rst), np.flatnonzero(st != rst)[:8]
    flagged = rst != 0
    assert np.isnan(Y[flagged]).all()
    err = np.abs(Y[~flagged].astype(np.float64) - ref[~flagged])
    cv = cond[~flagged]
    bad = err > RTOL * cv + ABS_FLOOR
    assert not bad.any(), (int(bad.sum()), float(err[bad].max()))
    pos = cv > 0
    return float((err[pos] / cv[pos]).max()) if pos.any() else 0.0


@pytest.mark.parametrize("case", load_golden("recurrent_hand.json")["cases"],
                         ids=lambda c: c["name"])
def test_hand_cases_exact(case):
    pop = population_from_rows([(case["nodes"], case["conns"])], case["n_in"], case["n_out"])
    X = np.array([case["x"]], np.float32)
    for T, want in case["outputs_by_T"].items():
        Y, st = gpu_recurrent(pop, X, int(T))
        assert st[0] == 0 and np.array_equal(Y[0, 0], np.array(want, np.float32)), (T, Y[0, 0])


def test_recurrent_tiles_and_tail():
    pop = synth.recurrent_population(P=96)
    obs = synth.normal_obs(96, 150, 17, 31)    # 2 full tiles + a tail of 22
    for T in (0, 1, 4, 10):
        Y, st = gpu_recurrent(pop, obs, T)
        if T == 0:
            assert (Y == 0).all()
        worst = check(pop, obs, T, Y, st)
        print(f"T={T}: worst |err|/cond {worst:.3e}")


def test_full_recurrent_workload():
    """Every genome of the 1000-genome recurrent workload, 1000 observations
    each, 10 sweeps (the bench's configuration)."""
    import oracle_pool
    pop = synth.recurrent_population()
    obs = synth.normal_obs(pop.P, oracle_pool.RECURRENT_B, pop.n_in,
                           synth.CONFIG_SEEDS["recurrent"] + 100)
    Y, st = gpu_recurrent(pop, obs, oracle_pool.RECURRENT_T)
    ref, cond, rst = oracle_pool.recurrent_reference(pop.P)
    worst = compare(Y, st, ref, cond, rst)
    print(f"recurrent workload: worst |err|/cond {worst:.3e} over {Y.size} outputs")


def test_acyclic_sum_genomes_give_forward_bits():
    import paper_2504_08339_amd as tn
    pop = synth.control_population(P=200)
    obs = synth.normal_obs(200, 70, 17, 9)
    depth = max(max(oracle.transform(oracle.decode(pop, g)).level.values())
                for g in range(pop.P))
    dp = to_device(pop)
    ff = host(tn.forward(dp, tn.transform(dp), tensor(obs)))
    Y = host(tn.forward_recurrent(dp, tensor(obs), depth + 1))
    sum_only = [g for g in range(pop.P) if (pop.node_agg[g][pop.node_key[g] >= 0] == 0).all()]
    assert len(sum_only) == pop.P
    assert np.array_equal(Y.view(np.uint32), ff.view(np.uint32))


def _random_cyclic(rng, n_in=3, n_out=2, n_hidden=7, n_conn=30):
    keys = list(range(n_in + n_out)) + [20 + h for h in range(n_hidden)]
    nodes = [[k, float(rng.normal()), float(rng.choice([1.0, 0.5, -0.75])),
              int(rng.integers(0, 7)), int(rng.integers(0, 6))] for k in keys]
    srcs, dsts = keys, [k for k in keys if k >= n_in]
    seen, conns = set(), []
    while len(conns) < n_conn:
        a, b = int(rng.choice(srcs)), int(rng.choice(dsts))
        if (a, b) not in seen:
            seen.add((a, b))
            conns.append([a, b, float(rng.normal() * 0.6), int(rng.random() < 0.85)])
    order = rng.permutation(len(nodes))
    return [nodes[i] for i in order], conns


def test_every_activation_and_aggregation():
    rng = np.random.default_rng(4)
    genomes = [_random_cyclic(rng) for _ in range(64)]
    pop = population_from_rows(genomes, 3, 2, N_max=16, C_max=40)
    obs = rng.normal(size=(64, 3)).astype(np.float32)
    for T in (1, 3, 7):
        Y, st = gpu_recurrent(pop, obs, T)
        check(pop, obs, T, Y, st)


def test_status_bits_and_ragged():
    io = [[0, 0, 1, 0, 0], [1, 0, 1, 0, 0]]
    genomes = [
        (io + [[5, 0.3, 1, 2, 0]], [[0, 5, 1.0, 1], [5, 5, 0.5, 1], [5, 1, 1.0, 1]]),
        (io, [[0, 7, 1.0, 1]]),                                          # dangling
        (io, [[0, 1, 1.0, 1], [0, 1, 2.0, 0]]),                          # repeated marking
        (io, [[1, 0, 1.0, 1]]),                                          # ends at an input
        ([io[0]], []),                                                   # missing output
        (io + [[5, 0, 1, 9, 0]], [[0, 5, 1.0, 1]]),                       # bad activation code
        (io + [[5, 0, 1, 0, 0], [5, 1, 1, 0, 0]], [[0, 5, 1.0, 1]]),     # repeated key
        (io + [[5, 0, 1, 0, 0]], [[0, 7, 1.0, 0], [5, 1, 1.0, 1]]),      # disabled dangling: fine
    ]
    pop = population_from_rows(genomes, 1, 1)
    obs = np.array([[0.5], [-2.0], [3.0]], np.float32)
    Y, st = gpu_recurrent(pop, obs, 5)
    check(pop, obs, 5, Y, st)
    rag = synth.to_ragged(pop)
    Yr, str_ = gpu_recurrent(rag, obs, 5)
    assert np.array_equal(str_, st)
    assert np.array_equal(Yr.view(np.uint32), Y.view(np.uint32))


def test_limits():
    import paper_2504_08339_amd as tn
    pop = synth.recurrent_population(P=4)
    dp = to_device(pop)
    obs = tensor(synth.normal_obs(4, 5, 17, 1))
    with pytest.raises(tn.TNError):
        tn.forward_recurrent(dp, obs, -1)
    big = population_from_rows([([[0, 0, 1, 0, 0], [1, 0, 1, 0, 0]], [[0, 1, 1.0, 1]])], 1, 1,
                               N_max=600, C_max=8)
    with pytest.raises(tn.TNError):
        tn.forward_recurrent(to_device(big), tensor(np.ones((3, 1), np.float32)), 2)
    Y = tn.forward_recurrent(dp, tensor(np.zeros((4, 0, 17), np.float32)), 3)
    assert Y.shape == (4, 0, 6)
