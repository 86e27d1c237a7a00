"""Pins of the oracle's calculation stage (TensorNEAT Section 3.3).

Checked against: hand-derived outputs of small networks (tests/golden), dense
linear algebra on layered genomes (NumPy matmul), and invariants that the
definition implies (disabled connections, dead-end nodes, key relabelling and
row permutation leave outputs unchanged). A last group plants mistakes into the
oracle and checks that the pins catch them.
"""
import numpy as np
import pytest

import oracle
import oracle.inference as of
import synth
from helpers import load_golden, mlp_genome, population_from_rows

GOLD = load_golden("hand_networks.json")


@pytest.mark.parametrize("case", GOLD["cases"], ids=[c["name"] for c in GOLD["cases"]])
def test_hand_networks(case):
    pop = population_from_rows([(case["nodes"], case["conns"])], case["n_in"], case["n_out"])
    X = np.array(case["obs"], np.float64)
    Y = oracle.forward_population(pop, X)[0]
    np.testing.assert_allclose(Y, np.array(case["expected"]), rtol=0, atol=case["tol"])
    if "expected_fitness" in case:
        f = oracle.xor_fitness(Y, synth.xor_targets())
        assert abs(f - case["expected_fitness"]) <= 4 * case["tol"] + 1e-15


@pytest.mark.parametrize("sizes,hidden_act,out_act", [
    ((17, 6), 0, 0),
    ((17, 6), 0, 2),
    ((4, 32, 2), 2, 0),
    ((5, 8, 7, 3), 1, 2),
    ((3, 4, 4, 4, 1), 4, 5),
])
def test_layered_genome_equals_matmul(sizes, hidden_act, out_act):
    rng = np.random.default_rng(sum(sizes))
    nodes, conns, Ws, bs = mlp_genome(rng, sizes, hidden_act, out_act)
    perm = rng.permutation(len(conns))          # row order must not matter beyond rounding
    conns = [conns[i] for i in perm]
    pop = population_from_rows([(nodes, conns)], sizes[0], sizes[-1])
    X = rng.standard_normal((50, sizes[0]))
    Y = oracle.forward_population(pop, X)[0]
    acts = {0: lambda z: z, 1: lambda z: 1 / (1 + np.exp(-z)), 2: np.tanh, 4: np.sin,
            5: lambda z: np.exp(-z * z)}
    h = X
    for l, (W, b) in enumerate(zip(Ws, bs)):
        a = acts[out_act if l == len(Ws) - 1 else hidden_act]
        h = a(h @ W.astype(np.float64) + b.astype(np.float64))
    np.testing.assert_allclose(Y, h, rtol=1e-12, atol=1e-12)


def test_response_and_bias_of_inputs():
    rng = np.random.default_rng(3)
    nodes, conns, Ws, bs = mlp_genome(rng, (3, 2), 0, 0, resp=-1.5)
    pop = population_from_rows([(nodes, conns)], 3, 2)
    X = rng.standard_normal((7, 3))
    Y = oracle.forward_population(pop, X)[0]
    np.testing.assert_allclose(Y, bs[0] + -1.5 * (X @ Ws[0].astype(np.float64)),
                               rtol=1e-13, atol=1e-13)


def _control(P=30):
    return synth.control_population(P=P)


def test_disabled_weights_have_no_effect():
    pop = _control()
    X = synth.normal_obs(pop.P, 16, 17, 9)
    Y = oracle.forward_population(pop, X)
    pop2 = synth.subset(pop, range(pop.P))
    off = (pop2.conn_en == 0) & (pop2.conn_in >= 0)
    assert off.any()
    pop2.conn_w[off] = 1e6
    assert np.array_equal(oracle.forward_population(pop2, X), Y)


def test_dead_end_node_has_no_effect():
    pop = _control(10)
    X = synth.normal_obs(pop.P, 8, 17, 11)
    Y = oracle.forward_population(pop, X)
    pop2 = synth.subset(pop, range(pop.P))
    for g in range(pop.P):
        nr = int(np.count_nonzero(pop2.node_key[g] >= 0))
        cr = int(np.count_nonzero(pop2.conn_in[g] >= 0))
        pop2.node_key[g, nr] = 100000
        pop2.node_bias[g, nr] = 0.3
        pop2.node_act[g, nr] = 1
        pop2.conn_in[g, cr], pop2.conn_out[g, cr], pop2.conn_w[g, cr], pop2.conn_en[g, cr] = 0, 100000, 5.0, 1
    assert np.array_equal(oracle.forward_population(pop2, X), Y)


def test_hidden_key_relabel_and_node_row_permutation_bitwise():
    pop = _control()
    X = synth.normal_obs(pop.P, 8, 17, 12)
    Y = oracle.forward_population(pop, X)
    relabel = synth.subset(pop, range(pop.P))
    n_io = pop.n_in + pop.n_out
    for arr in (relabel.node_key, relabel.conn_in, relabel.conn_out):
        hid = arr >= n_io
        arr[hid] = 7919 * arr[hid] + 13
    assert np.array_equal(oracle.forward_population(relabel, X), Y)
    perm = synth.permute_rows(pop, np.random.default_rng(5), nodes=True, conns=False)
    assert np.array_equal(oracle.forward_population(perm, X), Y)
    cperm = synth.permute_rows(pop, np.random.default_rng(6), nodes=False, conns=True)
    np.testing.assert_allclose(oracle.forward_population(cperm, X), Y, rtol=1e-12, atol=1e-12)


def test_flagged_genome_gives_nan():
    nodes = [[0, 0, 1, 0, 0], [1, 0, 1, 0, 0], [5, 0, 1, 0, 0], [6, 0, 1, 0, 0]]
    conns = [[0, 5, 1, 1], [5, 6, 1, 1], [6, 5, 1, 1], [6, 1, 1, 1]]
    pop = population_from_rows([(nodes, conns)], 1, 1)
    assert np.isnan(oracle.forward_population(pop, np.ones((3, 1)))).all()


def test_tolerance_scale_admits_float32_and_rejects_small_mistakes():
    """The parity tolerance |y - y64| <= 1e-5 * cond admits a float32 evaluation of
    the same definition (every step rounded), but not a bias off by 1e-3."""
    pop = synth.control_population(P=60)
    X = synth.normal_obs(pop.P, 64, 17, 13)
    worst = 0.0
    caught = 0
    for g in range(pop.P):
        gen = oracle.decode(pop, g)
        tr = oracle.transform(gen)
        Y64, cond = oracle.forward(gen, tr, X[g], with_cond=True)
        Y32 = oracle.forward(gen, tr, X[g], dtype=np.float32)
        err = np.abs(Y32 - Y64)
        assert np.all(err[cond == 0] == 0)
        pos = cond > 0
        worst = max(worst, float(np.max(err[pos] / cond[pos], initial=0.0)))
        out = gen.nodes[gen.n_in]
        out.bias += 1e-3
        Ybad = oracle.forward(gen, tr, X[g])
        caught += bool(np.any(np.abs(Ybad - Y64) > 1e-5 * cond))
    assert worst < 1e-6, worst          # float32 error well inside the 1e-5 budget
    assert caught == pop.P


# ---- planted mistakes: the pins above must fail -------------------------------

def _mlp_pin_fails(monkeypatch, patch):
    with monkeypatch.context() as m:
        patch(m)
        try:
            test_layered_genome_equals_matmul((5, 8, 7, 3), 1, 2)
        except AssertionError:
            return True
    return False


def test_planted_dropped_term(monkeypatch):
    orig = of.aggregate
    assert _mlp_pin_fails(monkeypatch, lambda m: m.setattr(
        of, "aggregate", lambda n, t, b, d=np.float64: orig(n, t[:-1], b, d)))


def test_planted_sign_error(monkeypatch):
    orig = of.activate
    assert _mlp_pin_fails(monkeypatch, lambda m: m.setattr(
        of, "activate", lambda n, z: orig(n, -z) if n == "tanh" else orig(n, z)))


def test_planted_wrong_source(monkeypatch):
    orig = oracle.genome.transform

    def shifted(gen):
        tr = orig(gen)
        for k, edges in tr.in_edges.items():
            if len(edges) > 1:
                tr.in_edges[k] = [oracle.genome.Conn(e.row, edges[0].kin, e.kout, e.w, e.enabled)
                                  for e in edges]
        return tr
    assert _mlp_pin_fails(monkeypatch, lambda m: m.setattr(of, "transform", shifted))


@pytest.mark.parametrize("name", ["sigmoid", "tanh"])
def test_activation_slope_bound_far_out(name):
    """The error-scale slope bound of sigmoid and tanh equals the largest |act'|
    over the interval, also far from 0 where act' is tiny but positive;
    references: exp(log_expit(x) + log_expit(-x)) (SciPy) and 1 / cosh(x)^2."""
    from scipy.special import log_expit
    ref = {"sigmoid": lambda x: np.exp(log_expit(x) + log_expit(-x)),
           "tanh": lambda x: 1.0 / np.cosh(x) ** 2}[name]
    from oracle.inference import activation_slope
    for z in np.linspace(-60.0, 60.0, 97):
        for r in (0.0, 0.1, 5.0):
            bound = float(activation_slope(name, np.array(z), np.array(r)))
            grid = np.linspace(z - r, z + r, 201)
            brute = float(ref(grid).max())
            assert bound >= brute * (1 - 1e-9), (z, r, bound, brute)
            assert bound <= ref(max(abs(z) - r, 0.0)) * (1 + 1e-9), (z, r)
            assert bound > 0.0
