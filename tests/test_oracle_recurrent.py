"""Pins of the oracle's recurrent forward pass (synchronous sweeps; reading in
oracle/recurrent.py).

* hand-worked cyclic networks (tests/golden/recurrent_hand.json);
* on acyclic genomes, T = the largest topological level + 1 gives the
  feedforward oracle's outputs bit for bit (the feedforward oracle is pinned on
  its own);
* with identity activations and sum aggregation the sweeps are the affine
  iteration v_t = A v_{t-1} + c, whose value after T steps, sum_{t<T} A^t c,
  NumPy's matrix power gives independently;
* invariants (row permutation, hidden-key relabelling, disabled connections)
  and status bits (cycles allowed, everything else flagged);
* planted mistakes (in-place sweeps, NaN start values, one sweep too many)
  fail the pins above.
"""
import numpy as np
import pytest

import oracle
import oracle.recurrent as orc
import synth
from helpers import load_golden, population_from_rows

GOLD = load_golden("recurrent_hand.json")


def _hand_genome(case):
    pop = population_from_rows([(case["nodes"], case["conns"])], case["n_in"], case["n_out"])
    return oracle.decode(pop, 0)


@pytest.mark.parametrize("case", GOLD["cases"], ids=lambda c: c["name"])
def test_hand_cases(case):
    gen = _hand_genome(case)
    X = np.array([case["x"]])
    for T, want in case["outputs_by_T"].items():
        y = oracle.recurrent_forward(gen, X, int(T))
        assert np.array_equal(y[0], np.array(want)), (T, y[0], want)


def test_acyclic_equals_feedforward_past_largest_level():
    pop = synth.control_population(P=40)
    X = synth.normal_obs(1, 16, pop.n_in, 7)[0]
    shorter_differs = 0
    for g in range(pop.P):
        gen = oracle.decode(pop, g)
        tr = oracle.transform(gen)
        assert tr.status == 0
        depth = max(tr.level.values())
        ff = oracle.forward(gen, tr, X)
        assert np.array_equal(oracle.recurrent_forward(gen, X, depth + 1), ff)
        assert np.array_equal(oracle.recurrent_forward(gen, X, depth + 4), ff)
        if depth >= 1 and not np.array_equal(oracle.recurrent_forward(gen, X, depth - 1), ff):
            shorter_differs += 1
    assert shorter_differs >= pop.P // 2


def _random_cyclic(rng, n_in=3, n_out=2, n_hidden=6, n_conn=24, identity=True):
    keys = list(range(n_in + n_out)) + [10 + h for h in range(n_hidden)]
    nodes = []
    for k in keys:
        act = 0 if identity else int(rng.choice([0, 1, 2, 3]))
        nodes.append([k, float(rng.normal()), float(rng.choice([1.0, 0.5, -0.75])), act, 0])
    srcs = [k for k in keys if not (n_in <= k < n_in + n_out)] + list(range(n_in, n_in + n_out))
    dsts = [k for k in keys if k >= n_in]
    seen, conns = set(), []
    while len(conns) < n_conn:
        a, b = int(rng.choice(srcs)), int(rng.choice(dsts))
        if (a, b) in seen:
            continue
        seen.add((a, b))
        conns.append([a, b, float(rng.normal() * 0.4), int(rng.random() < 0.85)])
    order = rng.permutation(len(nodes))
    return [nodes[i] for i in order], conns


def test_linear_networks_match_matrix_powers():
    rng = np.random.default_rng(5)
    for trial in range(20):
        nodes, conns = _random_cyclic(rng)
        pop = population_from_rows([(nodes, conns)], 3, 2)
        gen = oracle.decode(pop, 0)
        hid = sorted(k for k in gen.nodes if k >= 3)
        idx = {k: i for i, k in enumerate(hid)}
        A = np.zeros((len(hid), len(hid)))
        Bm = np.zeros((len(hid), 3))
        for c in gen.conns:
            if not c.enabled:
                continue
            rho = gen.nodes[c.kout].resp
            if c.kin < 3:
                Bm[idx[c.kout], c.kin] += rho * c.w
            else:
                A[idx[c.kout], idx[c.kin]] += rho * c.w
        bias = np.array([gen.nodes[k].bias for k in hid])
        X = rng.normal(size=(5, 3))
        for T in (0, 1, 2, 5, 9):
            y = oracle.recurrent_forward(gen, X, T)
            for b in range(5):
                c = bias + Bm @ X[b]
                vT = sum((np.linalg.matrix_power(A, t) @ c for t in range(T)), np.zeros(len(hid)))
                want = np.array([vT[idx[3]], vT[idx[4]]])
                assert np.allclose(y[b], want, rtol=1e-10, atol=1e-12), (trial, T, b)


def test_invariants():
    rng = np.random.default_rng(8)
    for _ in range(10):
        nodes, conns = _random_cyclic(rng, identity=False)
        X = rng.normal(size=(4, 3))
        base = oracle.recurrent_forward(oracle.decode(population_from_rows([(nodes, conns)], 3, 2), 0), X, 6)
        perm = [nodes[i] for i in rng.permutation(len(nodes))]
        relabel = {k: k + 100 for k in range(10, 16)}
        rn = [[relabel.get(n[0], n[0])] + n[1:] for n in nodes]
        rc = [[relabel.get(c[0], c[0]), relabel.get(c[1], c[1])] + c[2:] for c in conns]
        extra = conns + [[0, 3, 123.0, 0]] if not any(c[:2] == [0, 3] for c in conns) else conns
        for ns, cs in ((perm, conns), (rn, rc), (nodes, extra)):
            y = oracle.recurrent_forward(
                oracle.decode(population_from_rows([(ns, cs)], 3, 2), 0), X, 6)
            assert np.array_equal(y, base)


def test_status_bits():
    io = [[0, 0, 1, 0, 0], [1, 0, 1, 0, 0]]
    genomes = [
        (io + [[5, 0, 1, 0, 0]], [[0, 5, 1.0, 1], [5, 5, 1.0, 1], [5, 1, 1.0, 1]]),  # cyclic: fine
        (io, [[0, 7, 1.0, 1]]),                                                   # dangling
        (io, [[0, 1, 1.0, 1], [0, 1, 2.0, 0]]),                                   # repeated marking
        (io, [[1, 0, 1.0, 1]]),                                                   # ends at input
        ([io[0]], []),                                                            # missing output
    ]
    pop = population_from_rows(genomes, 1, 1)
    X = np.ones((2, 1))
    Y, st = orc.recurrent_population(pop, X, 4)
    assert list(st) == [0, oracle.DANGLING, oracle.DUP_CONN, oracle.INPUT_DST, oracle.MISSING_IO]
    assert np.isfinite(Y[0]).all() and np.isnan(Y[1:]).all()


# ---- planted mistakes --------------------------------------------------------

def _in_place_sweep(gen, edges, v, cond, B, dtype, with_cond):
    v = dict(v)
    for k in sorted(gen.nodes, key=lambda k: gen.nodes[k].row):
        node = gen.nodes[k]
        if k < gen.n_in:
            continue
        terms = [dtype(c.w) * v[c.kin] for c in edges[k]]
        s = oracle.aggregate(node.agg, terms, B, dtype)
        v[k] = oracle.activate(node.act, dtype(node.bias) + dtype(node.resp) * s)
    return v, cond


def _hand_pins_pass():
    try:
        for case in GOLD["cases"]:
            test_hand_cases(case)
        test_linear_networks_match_matrix_powers()
    except AssertionError:
        return False
    return True


def test_pins_pass_unplanted():
    assert _hand_pins_pass()


def test_planted_in_place_sweep_is_caught(monkeypatch):
    monkeypatch.setattr(orc, "_sweep", _in_place_sweep)
    assert not _hand_pins_pass()


def test_planted_nan_start_is_caught(monkeypatch):
    real = orc._sweep
    state = {"first": True}

    def nan_start(gen, edges, v, cond, B, dtype, with_cond):
        if state["first"]:
            state["first"] = False
            v = {k: (x if k < gen.n_in else np.full(B, np.nan)) for k, x in v.items()}
        return real(gen, edges, v, cond, B, dtype, with_cond)

    monkeypatch.setattr(orc, "_sweep", nan_start)
    assert not _hand_pins_pass()


def test_planted_extra_sweep_is_caught(monkeypatch):
    real = orc._sweep

    def twice(gen, edges, v, cond, B, dtype, with_cond):
        v, cond = real(gen, edges, v, cond, B, dtype, with_cond)
        return real(gen, edges, v, cond, B, dtype, with_cond)

    monkeypatch.setattr(orc, "_sweep", twice)
    assert not _hand_pins_pass()
