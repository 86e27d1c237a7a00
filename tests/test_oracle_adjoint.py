"""Pins of the oracle's reverse-mode gradient.

Checked against float64 central finite differences (h = 1e-6) of the oracle's
own forward on perturbed parameters, against torch's CPU float64 autograd on
layered genomes (a library routine that shares nothing with the oracle), and
against exact zeros for disabled and padding rows.
"""
import copy

import numpy as np
import pytest
import torch

import oracle
import synth
from helpers import mlp_genome, population_from_rows

H = 1e-6


def _loss(gen, tr, X, T):
    Y = oracle.forward(gen, tr, X)
    return float(np.mean((Y - T) ** 2))


def _fd_check(gen, X, T, max_params=None, rng=None):
    tr = oracle.transform(gen)
    Y = oracle.forward(gen, tr, X)
    dY = 2.0 * (Y - T) / Y.size
    dW, db = oracle.backward(gen, tr, X, dY)
    params = [("w", i) for i, c in enumerate(gen.conns) if c.enabled]
    params += [("b", k) for k in gen.nodes if k >= gen.n_in]
    if max_params is not None and len(params) > max_params:
        params = [params[i] for i in rng.choice(len(params), max_params, replace=False)]
    checked = 0
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
        fd = (_loss(gp, oracle.transform(gp), X, T) - _loss(gm, oracle.transform(gm), X, T)) / (2 * H)
        assert abs(g - fd) <= 1e-4 * abs(fd) + 1e-8, (kind, ident, g, fd)
        checked += 1
    return checked


def test_fd_differentiation_population():
    pop = synth.differentiation_population(P=12)
    X = synth.uniform_inputs(64, 4, 104)
    T = synth.target_mlp(X, 32, 2, 204).astype(np.float64)
    n = 0
    for g in range(pop.P):
        n += _fd_check(oracle.decode(pop, g), X, T)
    assert n > 200


@pytest.mark.parametrize("agg", [0, 1, 2, 3, 4, 5])
def test_fd_all_aggregations_and_activations(agg):
    rng = np.random.default_rng(10 + agg)
    pop = synth.cppn_population(P=6, seed=30 + agg)
    pop.node_agg[pop.node_key >= pop.n_in] = agg
    # mix every activation except the kinked relu / abs over non-input nodes
    acts = np.array([0, 1, 2, 4, 5], np.uint8)
    pop.node_act[:] = acts[rng.integers(len(acts), size=pop.node_act.shape)]
    X = rng.uniform(-1, 1, size=(16, pop.n_in))
    for g in range(pop.P):
        gen = oracle.decode(pop, g)
        T = np.zeros((16, pop.n_out))
        _fd_check(gen, X, T, max_params=40, rng=rng)


@pytest.mark.parametrize("sizes,hidden_act", [((4, 32, 2), 2), ((3, 5, 6, 2), 1), ((6, 3), 2)])
def test_torch_autograd_layered(sizes, hidden_act):
    rng = np.random.default_rng(sum(sizes))
    nodes, conns, Ws, bs = mlp_genome(rng, sizes, hidden_act, 0)
    pop = population_from_rows([(nodes, conns)], sizes[0], sizes[-1])
    X = rng.uniform(-1, 1, size=(40, sizes[0]))
    T = rng.standard_normal((40, sizes[-1]))
    Wt = [torch.tensor(W, dtype=torch.float64, requires_grad=True) for W in Ws]
    bt = [torch.tensor(b, dtype=torch.float64, requires_grad=True) for b in bs]
    h = torch.tensor(X)
    acts = {1: torch.sigmoid, 2: torch.tanh}
    for l in range(len(Wt)):
        h = h @ Wt[l] + bt[l]
        if l < len(Wt) - 1:
            h = acts[hidden_act](h)
    loss = torch.mean((h - torch.tensor(T)) ** 2)
    loss.backward()
    gen = oracle.decode(pop, 0)
    tr = oracle.transform(gen)
    Y = oracle.forward(gen, tr, X)
    dW, db = oracle.backward(gen, tr, X, 2.0 * (Y - T) / Y.size)
    # map connection (in-key, out-key) and node key back to dense indices
    keys = [list(range(sizes[0]))]
    nxt = sizes[0] + sizes[-1]
    for hsz in sizes[1:-1]:
        keys.append(list(range(nxt, nxt + hsz)))
        nxt += hsz
    keys.append(list(range(sizes[0], sizes[0] + sizes[-1])))
    for c in gen.conns:
        l = next(l for l in range(1, len(keys)) if c.kout in keys[l])
        i, j = keys[l - 1].index(c.kin), keys[l].index(c.kout)
        assert dW[c.row] == pytest.approx(Wt[l - 1].grad[i, j].item(), rel=1e-10, abs=1e-13)
    for k, n in gen.nodes.items():
        if k < sizes[0]:
            assert db[n.row] == 0.0
            continue
        l = next(l for l in range(1, len(keys)) if k in keys[l])
        assert db[n.row] == pytest.approx(bt[l - 1].grad[keys[l].index(k)].item(),
                                          rel=1e-10, abs=1e-13)


def test_disabled_and_padding_rows_get_zero():
    pop = synth.differentiation_population(P=10)
    X = synth.uniform_inputs(32, 4, 104)
    dY = np.random.default_rng(1).standard_normal((pop.P, 32, 2))
    dW, db = oracle.backward_population(pop, X, dY)
    dead = (pop.conn_in < 0) | (pop.conn_en == 0)
    assert np.all(dW[dead] == 0.0)
    assert np.all(db[pop.node_key < 0] == 0.0)
    assert np.all(db[(pop.node_key >= 0) & (pop.node_key < pop.n_in)] == 0.0)
