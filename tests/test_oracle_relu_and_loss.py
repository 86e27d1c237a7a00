"""Pins of the oracle's relu / abs derivatives and of its squared-error loss.

* Hand-derived gradients at the kinks (tests/golden/kinks_and_losses.json): the
  reading relu'(0) = abs'(0) = 0.
* Float64 central finite differences (h = 1e-6) on genomes whose hidden nodes
  use relu and abs; a parameter whose +-h perturbation moves any relu / abs
  pre-activation across 0 is excluded and counted (the derivative does not
  exist there).
* torch's CPU float64 autograd on layered relu and abs genomes (a library
  routine that shares nothing with the oracle).
* Hand-computed squared-error losses for sse_loss and xor_fitness.
A last group plants mistakes (relu' = 1 everywhere, the loss without the
square) and checks that these pins catch them.
"""
import copy

import numpy as np
import pytest
import torch

import oracle
import oracle.adjoint as oa
import synth
from helpers import load_golden, mlp_genome, population_from_rows

GOLD = load_golden("kinks_and_losses.json")
H = 1e-6
KINKED = ("relu", "abs")


@pytest.mark.parametrize("case", GOLD["gradients"], ids=[c["name"] for c in GOLD["gradients"]])
def test_kink_gradients_by_hand(case):
    pop = population_from_rows([(case["nodes"], case["conns"])], case["n_in"], case["n_out"])
    gen = oracle.decode(pop, 0)
    tr = oracle.transform(gen)
    dW, db = oracle.backward(gen, tr, np.array(case["obs"]), np.array(case["dY"]))
    for r, want in enumerate(case["expected_dW"]):
        assert dW[r] == want, (r, dW[r], want)
    for r, want in enumerate(case["expected_db"]):
        assert db[r] == want, (r, db[r], want)


@pytest.mark.parametrize("case", GOLD["losses"], ids=[c["name"] for c in GOLD["losses"]])
def test_losses_by_hand(case):
    got = oracle.sse_loss(np.array(case["Y"]), np.array(case["T"]), case["scale"], case["offset"])
    assert got == pytest.approx(case["expected"], rel=1e-15, abs=1e-15)
    if case["offset"] == 4.0 and case["scale"] == -1.0:
        assert oracle.xor_fitness(np.array(case["Y"]), np.array(case["T"])) == pytest.approx(
            case["expected"], rel=1e-15, abs=1e-15)


def _kink_signs(gen, X):
    tr = oracle.transform(gen)
    _, z_of, _ = oracle.forward(gen, tr, X, keep_values=True)
    return {k: np.sign(z) for k, z in z_of.items() if gen.nodes[k].act in KINKED}


def _loss(gen, X, T):
    Y = oracle.forward(gen, oracle.transform(gen), X)
    return float(np.mean((Y - T) ** 2))


def _fd_kinked(gen, X, T, rng, max_params=60):
    """(checked, excluded) parameters of one genome."""
    tr = oracle.transform(gen)
    Y = oracle.forward(gen, tr, X)
    dW, db = oracle.backward(gen, tr, X, 2.0 * (Y - T) / Y.size)
    params = [("w", i) for i, c in enumerate(gen.conns) if c.enabled]
    params += [("b", k) for k in gen.nodes if k >= gen.n_in]
    if len(params) > max_params:
        params = [params[i] for i in rng.choice(len(params), max_params, replace=False)]
    base = _kink_signs(gen, X)
    checked = excluded = 0
    for kind, ident in params:
        gp, gm = copy.deepcopy(gen), copy.deepcopy(gen)
        if kind == "w":
            gp.conns[ident].w += H
            gm.conns[ident].w -= H
            g = dW[gen.conns[ident].row]
        else:
            gp.nodes[ident].bias += H
            gm.nodes[ident].bias -= H
            g = db[gen.nodes[ident].row]
        sp, sm = _kink_signs(gp, X), _kink_signs(gm, X)
        if any(np.any(sp[k] != base[k]) or np.any(sm[k] != base[k]) or np.any(base[k] == 0)
               for k in base):
            excluded += 1
            continue
        fd = (_loss(gp, X, T) - _loss(gm, X, T)) / (2 * H)
        assert abs(g - fd) <= 1e-4 * abs(fd) + 1e-8, (kind, ident, g, fd)
        checked += 1
    return checked, excluded


def _relu_abs_population(P, seed, acts):
    pop = synth.control_population(P=P, seed=seed)
    rng = np.random.default_rng(seed)
    hidden = pop.node_key >= pop.n_in + pop.n_out
    pop.node_act[hidden] = np.array(acts, np.uint8)[rng.integers(len(acts), size=hidden.sum())]
    return pop


@pytest.mark.parametrize("acts", [(3,), (6,), (3, 6, 2)], ids=["relu", "abs", "mixed"])
def test_fd_relu_and_abs(acts):
    pop = _relu_abs_population(10, 40 + len(acts), acts)
    rng = np.random.default_rng(7)
    X = synth.normal_obs(pop.P, 24, pop.n_in, 77)
    checked = excluded = 0
    for g in range(pop.P):
        gen = oracle.decode(pop, g)
        assert any(n.act in KINKED for k, n in gen.nodes.items() if k >= gen.n_in)
        c, e = _fd_kinked(gen, X[g], np.zeros((24, pop.n_out)), rng)
        checked += c
        excluded += e
    # most perturbations stay on one side of every kink
    assert checked > 200 and excluded < checked, (checked, excluded)


@pytest.mark.parametrize("sizes,hidden_act", [((4, 16, 2), 3), ((3, 6, 5, 2), 3), ((5, 7, 3), 6)])
def test_torch_autograd_relu_abs(sizes, hidden_act):
    rng = np.random.default_rng(100 + sum(sizes))
    nodes, conns, Ws, bs = mlp_genome(rng, sizes, hidden_act, 0)
    pop = population_from_rows([(nodes, conns)], sizes[0], sizes[-1])
    X = rng.uniform(-1, 1, size=(40, sizes[0]))
    T = rng.standard_normal((40, sizes[-1]))
    Wt = [torch.tensor(W, dtype=torch.float64, requires_grad=True) for W in Ws]
    bt = [torch.tensor(b, dtype=torch.float64, requires_grad=True) for b in bs]
    act = {3: torch.relu, 6: torch.abs}[hidden_act]
    h = torch.tensor(X)
    for l in range(len(Wt)):
        h = h @ Wt[l] + bt[l]
        if l < len(Wt) - 1:
            h = act(h)
    loss = torch.mean((h - torch.tensor(T)) ** 2)
    loss.backward()
    gen = oracle.decode(pop, 0)
    tr = oracle.transform(gen)
    Y = oracle.forward(gen, tr, X)
    dW, db = oracle.backward(gen, tr, X, 2.0 * (Y - T) / Y.size)
    keys = [list(range(sizes[0]))]
    nxt = sizes[0] + sizes[-1]
    for hsz in sizes[1:-1]:
        keys.append(list(range(nxt, nxt + hsz)))
        nxt += hsz
    keys.append(list(range(sizes[0], sizes[0] + sizes[-1])))
    for c in gen.conns:
        l = next(l for l in range(1, len(keys)) if c.kout in keys[l])
        i, j = keys[l - 1].index(c.kin), keys[l].index(c.kout)
        want = Wt[l - 1].grad[i, j].item()
        assert dW[c.row] == pytest.approx(want, rel=1e-10, abs=1e-13)
    for k, n in gen.nodes.items():
        if k < sizes[0]:
            continue
        l = next(l for l in range(1, len(keys)) if k in keys[l])
        want = bt[l - 1].grad[keys[l].index(k)].item()
        assert db[n.row] == pytest.approx(want, rel=1e-10, abs=1e-13)
    # both branches of the derivative are exercised: the first hidden layer's
    # pre-activations take both signs
    z1 = X @ Ws[0].astype(np.float64) + bs[0].astype(np.float64)
    assert 0.1 < np.mean(z1 < 0) < 0.9


# ---- planted mistakes: the pins above must fail -------------------------------

def _fails(fn, *args):
    try:
        fn(*args)
    except AssertionError:
        return True
    return False


def test_planted_relu_derivative_one(monkeypatch):
    orig = oa.activation_derivative

    def wrong(name, z):
        return np.ones_like(z) if name == "relu" else orig(name, z)
    with monkeypatch.context() as m:
        m.setattr(oa, "activation_derivative", wrong)
        assert _fails(test_torch_autograd_relu_abs, (4, 16, 2), 3)
        assert _fails(test_fd_relu_and_abs, (3,))
        assert _fails(test_kink_gradients_by_hand, GOLD["gradients"][0])


def test_planted_relu_kink_value(monkeypatch):
    orig = oa.activation_derivative

    def wrong(name, z):
        return (z >= 0.0).astype(np.float64) if name == "relu" else orig(name, z)
    with monkeypatch.context() as m:
        m.setattr(oa, "activation_derivative", wrong)
        assert _fails(test_kink_gradients_by_hand, GOLD["gradients"][0])


def test_planted_sse_without_square(monkeypatch):
    def wrong(Y, T, scale=1.0, offset=0.0):
        d = np.asarray(Y, np.float64) - np.asarray(T, np.float64)
        return offset + scale * float(np.sum(np.abs(d)))
    with monkeypatch.context() as m:
        m.setattr(oracle, "sse_loss", wrong)
        assert all(_fails(test_losses_by_hand, c) for c in GOLD["losses"])
