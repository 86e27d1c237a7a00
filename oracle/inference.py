"""The calculation stage of tensorized network inference (TensorNEAT Section 3.3).

TEST INFRASTRUCTURE ONLY (see the package docstring).

For one genome and a batch of observations, in float64:

* input node values are the observation components, v[key i] = x[i] (the paper
  sets v[k_input] to the inputs; their bias and activation are not applied);
* every other node, in topological order, takes
      s = agg(w_e * v[src_e] for its enabled in-edges, ascending connection row)
      z = b + rho * s
      v = act(z)
  which is f_n(f_c(.)) of Section 3.3 with f_c = w * input and
  f_n = act(agg + b). Reading: the node response rho (a node hyperparameter in
  Appendix A) scales the aggregate; with rho = 1, as in the paper's experiments
  (Appendix C), this is exactly the printed rule;
* outputs are v[key I + j].

Readings: missing expanded connections (NaN in C_exp) are absent terms, never
multiplied; an aggregation over no terms is 0, so a node without enabled
in-edges outputs act(b). Activation functions, never defined in the paper,
follow their usual definitions: sigmoid 1/(1+e^-z) with no scaling, tanh, relu
max(0,z), sin, gaussian e^(-z^2), abs, identity.

``forward`` also returns a first-order error scale for each output, used by the
tests to turn the relative tolerance into an absolute one (``cond``): inputs
carry |x|; a node carries |v| + S * (|b| + |rho| * sum_e |w_e| * cond[src_e]),
where S bounds |act'| on a neighbourhood of z. Rounding errors of a float32
evaluation propagate through the same linearised sensitivities, so
|y32 - y64| stays a small multiple of the unit roundoff times cond.
"""
from __future__ import annotations

import math
from typing import List, Optional

import numpy as np

from .genome import decode, transform


def activate(name: str, z: np.ndarray) -> np.ndarray:
    if name == "identity":
        return z
    if name == "sigmoid":
        return 1.0 / (1.0 + np.exp(-z))
    if name == "tanh":
        return np.tanh(z)
    if name == "relu":
        return np.maximum(z, 0.0)
    if name == "sin":
        return np.sin(z)
    if name == "gaussian":
        return np.exp(-z * z)
    if name == "abs":
        return np.abs(z)
    raise ValueError(name)


def activation_derivative(name: str, z: np.ndarray) -> np.ndarray:
    """d act / dz; at the kinks of relu and abs the derivative taken is 0."""
    if name == "identity":
        return np.ones_like(z)
    if name == "sigmoid":
        s = 1.0 / (1.0 + np.exp(-z))
        return s * (1.0 - s)
    if name == "tanh":
        t = np.tanh(z)
        return 1.0 - t * t
    if name == "relu":
        return (z > 0.0).astype(np.float64)
    if name == "sin":
        return np.cos(z)
    if name == "gaussian":
        return -2.0 * z * np.exp(-z * z)
    if name == "abs":
        return np.sign(z)
    raise ValueError(name)


def activation_slope(name: str, z: np.ndarray, r: np.ndarray) -> np.ndarray:
    """Upper bound of |act'| over the interval [z - r, z + r]."""
    z = np.asarray(z, np.float64)
    r = np.asarray(r, np.float64) + np.zeros_like(z)
    if name in ("identity", "abs"):
        return np.ones_like(z)
    if name == "relu":
        return (z + r > 0.0).astype(np.float64)
    lo = np.maximum(np.abs(z) - r, 0.0)          # smallest |zeta| in the interval
    hi = np.abs(z) + r                           # largest |zeta|
    # both slopes peak at 0 and fall with |zeta|; written without 1 - s
    # (which rounds to 0 once s rounds to 1, from |zeta| of about 19 for tanh
    # and 37 for sigmoid, while the true slope is still positive)
    if name == "tanh":
        e = np.exp(-2.0 * lo)
        return 4.0 * e / ((1.0 + e) * (1.0 + e))
    if name == "sigmoid":
        e = np.exp(-lo)
        return e / ((1.0 + e) * (1.0 + e))
    if name == "sin":
        k_lo = np.ceil((z - r) / math.pi)
        k_hi = np.floor((z + r) / math.pi)
        ends = np.maximum(np.abs(np.cos(z - r)), np.abs(np.cos(z + r)))
        return np.where(k_hi >= k_lo, 1.0, ends)
    if name == "gaussian":
        f = lambda u: 2.0 * u * np.exp(-u * u)
        peak = 1.0 / math.sqrt(2.0)
        inside = (lo <= peak) & (peak <= hi)
        return np.where(inside, f(peak), np.maximum(f(lo), f(hi)))
    raise ValueError(name)


def aggregate(name: str, terms: List[np.ndarray], batch: int,
              dtype=np.float64) -> np.ndarray:
    """Aggregation over a node's incoming terms, in the listed order (empty -> 0)."""
    if not terms:
        return np.zeros(batch, dtype)
    if name == "sum":
        s = np.zeros(batch, dtype)
        for t in terms:
            s = s + t
        return s
    if name == "mean":
        s = np.zeros(batch, dtype)
        for t in terms:
            s = s + t
        return s / dtype(len(terms))
    if name == "product":
        s = np.ones(batch, dtype)
        for t in terms:
            s = s * t
        return s
    if name == "max":
        s = terms[0]
        for t in terms[1:]:
            s = np.maximum(s, t)
        return s
    if name == "min":
        s = terms[0]
        for t in terms[1:]:
            s = np.minimum(s, t)
        return s
    if name == "maxabs":
        s = terms[0]
        for t in terms[1:]:
            s = np.where(np.abs(t) > np.abs(s), t, s)
        return s
    raise ValueError(name)


def _term_magnitude(name: str, terms, term_scales, batch: int) -> np.ndarray:
    """First-order scale of agg's error from its terms' error scales."""
    if not terms:
        return np.zeros(batch)
    if name == "product":
        m = np.zeros(batch)
        for i, sc in enumerate(term_scales):
            p = sc.copy()
            for j, t in enumerate(terms):
                if j != i:
                    p = p * np.abs(t)
            m = m + p
        return m
    m = np.zeros(batch)
    for sc in term_scales:
        m = m + sc
    if name == "mean":
        m = m / len(terms)
    return m


def forward(gen, tr, X: np.ndarray, with_cond: bool = False, keep_values: bool = False,
            dtype=np.float64):
    """Outputs [B][O] of one decoded + transformed genome on X [B][I].

    A flagged genome (tr.status != 0) yields NaN outputs.
    With ``with_cond`` also returns the per-output error scale (see module doc).
    With ``keep_values`` also returns dicts key -> z and key -> v over the batch.
    ``dtype`` is float64 (the reference); float32 evaluates every step rounded to
    float32, which the tests use only to check the tolerance derivation.
    """
    X = np.asarray(X, dtype)
    B = X.shape[0]
    O = gen.n_out
    if tr.status:
        Y = np.full((B, O), np.nan)
        res = [Y]
        if with_cond:
            res.append(np.full((B, O), np.nan))
        if keep_values:
            res += [{}, {}]
        return res[0] if len(res) == 1 else tuple(res)
    v, z_of, cond = {}, {}, {}
    for k in tr.order:
        if k < gen.n_in:
            v[k] = X[:, k]
            cond[k] = np.abs(X[:, k])
            continue
        node = gen.nodes[k]
        edges = tr.in_edges[k]
        terms = [dtype(c.w) * v[c.kin] for c in edges]
        s = aggregate(node.agg, terms, B, dtype)
        z = dtype(node.bias) + dtype(node.resp) * s
        val = activate(node.act, z)
        v[k] = val
        z_of[k] = z
        if with_cond:
            assert dtype == np.float64
            scales = [abs(c.w) * cond[c.kin] for c in edges]
            m = _term_magnitude(node.agg, terms, scales, B)
            cz = abs(node.bias) + abs(node.resp) * m
            cond[k] = np.abs(val) + activation_slope(node.act, z, 1e-3 * cz) * cz
    Y = np.stack([v[gen.n_in + j] for j in range(O)], axis=1)
    res = [Y]
    if with_cond:
        res.append(np.stack([cond[gen.n_in + j] for j in range(O)], axis=1))
    if keep_values:
        res += [z_of, v]
    return res[0] if len(res) == 1 else tuple(res)


def forward_population(pop, obs: np.ndarray, genomes: Optional[List[int]] = None,
                       with_cond: bool = False):
    """Outputs [len(genomes)][B][O] for each listed genome.

    ``obs`` is [B][I] (shared by every genome) or [P][B][I] (per genome).
    """
    idx = list(range(pop.P)) if genomes is None else list(genomes)
    ys, cs = [], []
    for g in idx:
        gen = decode(pop, g)
        tr = transform(gen)
        X = obs if obs.ndim == 2 else obs[g]
        r = forward(gen, tr, X, with_cond=with_cond)
        if with_cond:
            ys.append(r[0])
            cs.append(r[1])
        else:
            ys.append(r)
    if with_cond:
        return np.stack(ys), np.stack(cs)
    return np.stack(ys)


def xor_fitness(Y: np.ndarray, T: np.ndarray) -> float:
    """Fitness 4 - sum of squared errors over the four XOR rows."""
    return 4.0 - float(np.sum((np.asarray(Y, np.float64) - np.asarray(T, np.float64)) ** 2))


def sse_loss(Y: np.ndarray, T: np.ndarray, scale: float = 1.0, offset: float = 0.0) -> float:
    """offset + scale * sum of squared errors; the MSE over B x O outputs is
    scale = 1/(B*O), the XOR fitness is offset 4, scale -1."""
    d = np.asarray(Y, np.float64) - np.asarray(T, np.float64)
    return offset + scale * float(np.sum(d * d))
