"""Forward pass of recurrent networks (network_type = recurrent, Appendix A).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper sorts networks into feedforward and recurrent ones by whether their
enabled connections form cycles (Section 3.3), and details the transformation
and calculation only for feedforward networks. A recurrent network has no
topological order, so the reading taken here evaluates it by synchronous
sweeps over all nodes:

* v_0: input nodes hold the observation (as in the feedforward rule, with no
  bias or activation); every other node starts at 0 (the paper's NaN start
  value would spread around a cycle and never leave it);
* sweep t = 1 .. T: every non-input node k takes
      v_t[k] = act_k(b_k + rho_k * agg_k(w_e * v_{t-1}[src_e]))
  over its enabled in-edges e in ascending connection row, every value on the
  right from the previous sweep (all nodes updated at once); inputs keep their
  values;
* outputs are v_T[key I + j]; with T = 0 they are the start values, 0.

The node rule, the aggregations over no terms (0), the activations and the
response term are those of the feedforward oracle (module ``inference``).
Genome checks are the transformation's (module ``genome``) except that a cycle
is allowed: a genome with a repeated key or marking, a dangling or
input-ending enabled connection, a missing input or output, a bad attribute
code, or oversize rows yields NaN outputs.

A consequence used as a pin: on an acyclic genome, a non-input node at level
L (longest enabled path from a node without in-edges) holds its feedforward
value from sweep L + 1 on (by induction: its sources are exact from sweep L,
inputs from sweep 0, and a node without in-edges takes act(b) in sweep 1), so
for T above the largest level the outputs equal the feedforward outputs
exactly (every value is computed by the same operations on the same
operands).
"""
from __future__ import annotations

from typing import Dict, List, Tuple

import numpy as np

from .genome import CYCLE, Conn, Genome, decode, transform
from .inference import activate, activation_slope, aggregate, _term_magnitude


def recurrent_status(gen: Genome) -> int:
    """The transformation's status bits with a cycle allowed (CYCLE is only
    reported when no other bit is set, so clearing it leaves the others)."""
    return transform(gen).status & ~CYCLE


def in_edges(gen: Genome) -> Dict[int, List[Conn]]:
    """Enabled in-edges of every node key, ascending connection row."""
    edges: Dict[int, List[Conn]] = {k: [] for k in gen.nodes}
    for c in gen.conns:
        if c.enabled:
            edges[c.kout].append(c)
    for k in edges:
        edges[k].sort(key=lambda c: c.row)
    return edges


def _sweep(gen: Genome, edges, v, cond, B: int, dtype, with_cond: bool):
    """One synchronous sweep: every non-input node from the previous values."""
    nv, nc = {}, {}
    for k, node in gen.nodes.items():
        if k < gen.n_in:
            nv[k], nc[k] = v[k], cond[k]
            continue
        terms = [dtype(c.w) * v[c.kin] for c in edges[k]]
        s = aggregate(node.agg, terms, B, dtype)
        z = dtype(node.bias) + dtype(node.resp) * s
        nv[k] = activate(node.act, z)
        if with_cond:
            scales = [abs(c.w) * cond[c.kin] for c in edges[k]]
            m = _term_magnitude(node.agg, terms, scales, B)
            cz = abs(node.bias) + abs(node.resp) * m
            nc[k] = np.abs(nv[k]) + activation_slope(node.act, z, 1e-3 * cz) * cz
    return nv, nc


def recurrent_forward(gen: Genome, X: np.ndarray, T: int, with_cond: bool = False,
                      dtype=np.float64):
    """Outputs [B][O] after T synchronous sweeps (module docstring). With
    ``with_cond`` also the first-order error scale of each output, propagated
    through the sweeps the same way the feedforward oracle propagates it
    through the topological order."""
    X = np.asarray(X, dtype)
    B, O = X.shape[0], gen.n_out
    if recurrent_status(gen):
        Y = np.full((B, O), np.nan)
        return (Y, np.full((B, O), np.nan)) if with_cond else Y
    edges = in_edges(gen)
    v = {k: (X[:, k] if k < gen.n_in else np.zeros(B, dtype)) for k in gen.nodes}
    cond = {k: (np.abs(X[:, k]) if k < gen.n_in else np.zeros(B)) for k in gen.nodes}
    for _ in range(T):
        v, cond = _sweep(gen, edges, v, cond, B, dtype, with_cond)
    Y = np.stack([v[gen.n_in + j] for j in range(O)], axis=1)
    if with_cond:
        return Y, np.stack([cond[gen.n_in + j] for j in range(O)], axis=1)
    return Y


def recurrent_population(pop, obs: np.ndarray, T: int, genomes=None, with_cond: bool = False):
    """recurrent_forward for each listed genome (obs [B][I] shared or [P][B][I]);
    also returns the status bits per genome."""
    idx = list(range(pop.P)) if genomes is None else list(genomes)
    ys, cs, st = [], [], []
    for g in idx:
        gen = decode(pop, g)
        X = obs if obs.ndim == 2 else obs[g]
        r = recurrent_forward(gen, X, T, with_cond=with_cond)
        if with_cond:
            ys.append(r[0])
            cs.append(r[1])
        else:
            ys.append(r)
        st.append(recurrent_status(gen))
    res: Tuple = (np.stack(ys),)
    if with_cond:
        res += (np.stack(cs),)
    return res + (np.array(st, np.int32),)
