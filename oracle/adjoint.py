"""Reverse-mode derivative of the calculation stage (gradient refinement of
weights; the paper's library evolves weights only, so this follows from the
forward rule of TensorNEAT Section 3.3 by the chain rule).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Given the upstream gradient dY = dL/dY [B][O] for one genome, walk the
topological order backwards. For node k with z = b + rho * agg(t_e),
t_e = w_e * v[src_e], v = act(z):

    gbar_k  = dL/dv_k (dY for an output key, plus what consumers send back)
    delta_k = gbar_k * act'(z_k)
    dL/db_k = sum over the batch of delta_k
    for each enabled in-edge e = (j -> k):
        dL/dt_e  = delta_k * rho_k * d agg / d t_e
        dL/dw_e += sum over the batch of dL/dt_e * v_j
        gbar_j  += dL/dt_e * w_e

d agg / d t_e is 1 for sum, 1/n for mean, the product of the other terms for
product, and for max / min / maxabs 1 at the first extreme term in row order
and 0 elsewhere. act' at the kinks of relu and abs is taken as 0.
Inputs have no bias gradient; disabled and padding rows get exactly 0.
"""
from __future__ import annotations

from typing import List, Optional

import numpy as np

from .inference import activation_derivative, forward
from .genome import decode, transform


def _agg_partials(name: str, terms: List[np.ndarray]) -> List[np.ndarray]:
    n = len(terms)
    if name == "sum":
        return [np.ones_like(t) for t in terms]
    if name == "mean":
        return [np.full_like(t, 1.0 / n) for t in terms]
    if name == "product":
        out = []
        for i in range(n):
            p = np.ones_like(terms[0])
            for j in range(n):
                if j != i:
                    p = p * terms[j]
            out.append(p)
        return out
    # max / min / maxabs: the first extreme term in row order takes the gradient
    if name == "max":
        key = lambda t: t
        better = lambda a, b: a > b
    elif name == "min":
        key = lambda t: t
        better = lambda a, b: a < b
    elif name == "maxabs":
        key = np.abs
        better = lambda a, b: a > b
    else:
        raise ValueError(name)
    best = np.zeros(terms[0].shape, np.int64)
    best_val = key(terms[0])
    for i in range(1, n):
        kv = key(terms[i])
        take = better(kv, best_val)
        best = np.where(take, i, best)
        best_val = np.where(take, kv, best_val)
    return [(best == i).astype(np.float64) for i in range(n)]


def backward(gen, tr, X: np.ndarray, dY: np.ndarray):
    """(dW, db): dW[conn row], db[node row] as dicts row -> float (only nonzero
    candidates listed); NaN-filled dicts are returned for a flagged genome."""
    X = np.asarray(X, np.float64)
    dY = np.asarray(dY, np.float64)
    if tr.status:
        return ({c.row: np.nan for c in gen.conns},
                {n.row: np.nan for n in gen.nodes.values()})
    _, z_of, v = forward(gen, tr, X, keep_values=True)
    B = X.shape[0]
    gbar = {k: np.zeros(B) for k in gen.nodes}
    for j in range(gen.n_out):
        gbar[gen.n_in + j] = gbar[gen.n_in + j] + dY[:, j]
    dW = {c.row: 0.0 for c in gen.conns}
    db = {n.row: 0.0 for n in gen.nodes.values()}
    for k in reversed(tr.order):
        if k < gen.n_in:
            continue
        node = gen.nodes[k]
        delta = gbar[k] * activation_derivative(node.act, z_of[k])
        db[node.row] = float(np.sum(delta))
        edges = tr.in_edges[k]
        if not edges:
            continue
        terms = [c.w * v[c.kin] for c in edges]
        partials = _agg_partials(node.agg, terms)
        for c, dp in zip(edges, partials):
            dt = delta * node.resp * dp
            dW[c.row] = float(np.sum(dt * v[c.kin]))
            gbar[c.kin] = gbar[c.kin] + dt * c.w
    return dW, db


def backward_population(pop, X: np.ndarray, dY: np.ndarray,
                        genomes: Optional[List[int]] = None):
    """Dense gradients: dW [len][C_max], db [len][N_max] (padded layout only).

    ``X`` is [B][I] shared or [P][B][I]; ``dY`` is [P][B][O] indexed by genome.
    """
    idx = list(range(pop.P)) if genomes is None else list(genomes)
    dW = np.zeros((len(idx), pop.C_max))
    db = np.zeros((len(idx), pop.N_max))
    for a, g in enumerate(idx):
        gen = decode(pop, g)
        tr = transform(gen)
        Xg = X if X.ndim == 2 else X[g]
        w, b = backward(gen, tr, Xg, dY[g])
        for r, val in w.items():
            dW[a, r] = val
        for r, val in b.items():
            db[a, r] = val
        if tr.status:
            dW[a, :] = np.nan
            db[a, :] = np.nan
    return dW, db
