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
