"""Compatibility distance for speciation (TensorNEAT Section 2.1, Algorithm 1's
"divide pop by distances between networks"; coefficients in Appendix A).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper names the distance and its coefficients but prints no formula, and
says its own distance differs from NEAT-Python's. Reading taken here: the
original NEAT compatibility distance over connection genes,

    delta = c1 * E / N + c2 * D / N + c3 * Wbar

* genes are all valid connection rows of a genome, enabled or not, identified by
  their historical marking (in-key, out-key);
* innovation order is lexicographic order of (in-key, out-key);
* matching genes M are markings present in both genomes;
* excess genes E are non-matching genes whose marking is beyond the smaller of
  the two genomes' largest markings (all genes of the other genome when one
  genome has none);
* disjoint genes D are the remaining non-matching genes;
* Wbar is the mean |w1 - w2| over matching genes (0 when there are none);
* N is the larger gene count; two empty genomes are at distance 0.

A genome holding two rows with the same marking, or a ragged genome above its
declared capacity, has no defined gene set: its distances are NaN and its
counts -1.
"""
from __future__ import annotations

import math
from typing import Dict, List, Optional, Tuple

import numpy as np

from .genome import OVERSIZE, decode


def genome_genes(pop, g: int) -> Optional[Dict[Tuple[int, int], float]]:
    """Marking -> weight for genome g, or None if a marking repeats."""
    gen = decode(pop, g)
    if gen.status & OVERSIZE:
        return None
    genes: Dict[Tuple[int, int], float] = {}
    for c in gen.conns:
        key = (c.kin, c.kout)
        if key in genes:
            return None
        genes[key] = float(np.float32(c.w))
    return genes


def distance(g1, g2, c1: float = 1.0, c2: float = 1.0, c3: float = 0.4):
    """(delta, E, D) between two gene dictionaries."""
    if g1 is None or g2 is None:
        return math.nan, -1, -1
    k1, k2 = set(g1), set(g2)
    if not k1 and not k2:
        return 0.0, 0, 0
    matching = k1 & k2
    non_matching = (k1 | k2) - matching
    if k1 and k2:
        limit = min(max(k1), max(k2))
        excess = sum(1 for k in non_matching if k > limit)
    else:
        excess = len(non_matching)
    disjoint = len(non_matching) - excess
    wbar = (sum(abs(g1[k] - g2[k]) for k in sorted(matching)) / len(matching)
            if matching else 0.0)
    n = max(len(k1), len(k2))
    return c1 * excess / n + c2 * disjoint / n + c3 * wbar, excess, disjoint


def distance_matrix(pop, c1: float = 1.0, c2: float = 1.0, c3: float = 0.4,
                    pairs: Optional[List[Tuple[int, int]]] = None):
    """Full P x P (delta, E, D) matrices, or per-pair arrays for a list of pairs."""
    genes = {}

    def get(g):
        if g not in genes:
            genes[g] = genome_genes(pop, g)
        return genes[g]

    if pairs is not None:
        out = [distance(get(i), get(j), c1, c2, c3) for i, j in pairs]
        return (np.array([o[0] for o in out]), np.array([o[1] for o in out]),
                np.array([o[2] for o in out]))
    P = pop.P
    dist = np.zeros((P, P))
    E = np.zeros((P, P), np.int64)
    D = np.zeros((P, P), np.int64)
    for i in range(P):
        for j in range(P):
            dist[i, j], E[i, j], D[i, j] = distance(get(i), get(j), c1, c2, c3)
    return dist, E, D


# ---------------------------------------------------------------------------
# Node-inclusive distance (the paper's own coefficient pair, Appendix A:
# compatibility_disjoint and compatibility_homologous; Section 5.2 notes that
# the library's distance differs from NEAT-Python's; its formula is not
# printed). Reading taken here, over node genes and connection genes alike:
#
#     delta = delta_nodes + delta_conns
#     delta_X = (c_d * D_X + c_h * H_X) / max(|X1|, |X2|)   (0 if both empty)
#
# * node genes: valid non-input node rows, identified by key (input nodes are
#   the same in every genome and carry no attribute the forward pass uses);
#   connection genes: valid connection rows, enabled or not, identified by
#   marking (in-key, out-key);
# * D_X: genes whose identity only one genome holds (non-homologous);
# * H_X: sum over homologous genes, in ascending identity order, of
#   |bias1 - bias2| + |resp1 - resp2| + [act1 != act2] + [agg1 != agg2] for
#   nodes and |w1 - w2| + [enabled1 != enabled2] for connections.
# A genome with a repeated key or marking (or above its declared capacity) has
# no gene set: its distances are NaN and its counts -1.
# ---------------------------------------------------------------------------

def node_genes(pop, g: int):
    """(nodes, conns): key -> (bias, resp, act, agg) over non-input node rows and
    marking -> (w, enabled) over connection rows; None if a key or marking repeats."""
    gen = decode(pop, g)
    if gen.status & OVERSIZE:
        return None
    nodes = {}
    seen = set()
    (key, bias, resp, act, agg), _ = _node_rows(pop, g)
    for r in range(key.shape[0]):
        k = int(key[r])
        if k < 0:
            continue
        if k in seen:
            return None
        seen.add(k)
        if k >= gen.n_in:
            nodes[k] = (float(np.float32(bias[r])), float(np.float32(resp[r])), int(act[r]),
                        int(agg[r]))
    conns = {}
    for c in gen.conns:
        m = (c.kin, c.kout)
        if m in conns:
            return None
        conns[m] = (float(np.float32(c.w)), bool(c.enabled))
    return nodes, conns


def _node_rows(pop, g):
    from .genome import _rows
    return _rows(pop, g)


def distance_nodes(a, b, c_d: float = 1.0, c_h: float = 0.5):
    """(delta, D_nodes, D_conns) between two node_genes() results."""
    if a is None or b is None:
        return math.nan, -1, -1
    total = 0.0
    counts = []
    for x, y, attr in ((a[0], b[0], _node_attr_distance), (a[1], b[1], _conn_attr_distance)):
        kx, ky = set(x), set(y)
        hom = kx & ky
        d = len(kx) + len(ky) - 2 * len(hom)
        counts.append(d)
        n = max(len(kx), len(ky))
        if n == 0:
            continue
        h = 0.0
        for k in sorted(hom):
            h += attr(x[k], y[k])
        total += (c_d * d + c_h * h) / n
    return total, counts[0], counts[1]


def _node_attr_distance(p, q):
    return abs(p[0] - q[0]) + abs(p[1] - q[1]) + (p[2] != q[2]) + (p[3] != q[3])


def _conn_attr_distance(p, q):
    return abs(p[0] - q[0]) + (p[1] != q[1])


def distance_nodes_matrix(pop, c_d: float = 1.0, c_h: float = 0.5,
                          pairs: Optional[List[Tuple[int, int]]] = None):
    """P x P (delta, D_nodes, D_conns), or per-pair arrays for a list of pairs."""
    genes = {}

    def get(g):
        if g not in genes:
            genes[g] = node_genes(pop, g)
        return genes[g]

    if pairs is not None:
        out = [distance_nodes(get(i), get(j), c_d, c_h) for i, j in pairs]
        return tuple(np.array([o[k] for o in out]) for k in range(3))
    P = pop.P
    dist = np.zeros((P, P))
    DN = np.zeros((P, P), np.int64)
    DC = np.zeros((P, P), np.int64)
    for i in range(P):
        for j in range(P):
            dist[i, j], DN[i, j], DC[i, j] = distance_nodes(get(i), get(j), c_d, c_h)
    return dist, DN, DC
