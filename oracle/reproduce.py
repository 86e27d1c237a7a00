"""Tensorized reproduction: crossover and mutation of padded genomes
(TensorNEAT Section 3.2, with the hyperparameters of Appendices A and C).

TEST INFRASTRUCTURE ONLY (see the package docstring).

A genome is its padded node rows and connection rows (Section 3.1). Every
structural change is one of the paper's three tensorized operations:

* node addition       N[r_i] <- n_new, r_i the first empty row;
* node removal        N[r_j] <- NaN (here: the row made empty);
* connection addition / removal, the same on C;
* attribute change    n[1 + j] <- attr'_j, c[3 + j] <- attr'_j.

Crossover and mutation are built from them, in this order for one child:

1. Crossover (NEAT's alignment by historical marking, Section 2.1): the child
   takes the fitter parent's rows as they are (same positions). A node row of
   that parent whose key the other parent also holds, and a connection row
   whose marking (in-key, out-key) the other parent also holds, takes the other
   parent's attributes (bias, response, act, agg; weight, enabled flag) when
   its coin is below 1/2. Genes of the less fit parent that the fitter one
   lacks are not inherited. Identical parents give the parent back.
2. Add node (probability node_add): an enabled connection a -> b is picked; it
   is disabled; a new node takes the first empty node row, with the key given
   for the marking (a, b) by the call's innovation table, its bias and
   response from their initial distributions, the default activation and
   aggregation; a -> new with weight 1 and new -> b with the old weight take
   the first two empty connection rows (original NEAT's split, which leaves
   the network's function unchanged for an identity node with bias 0).
   Nothing changes when a node row or two connection rows are missing.
3. Delete node (node_delete): a hidden node row is made empty together with
   every connection row that names its key.
4. Add connection (conn_add): a source among the input and hidden node rows
   and a destination among the hidden and output node rows are picked; the
   connection is added in the first empty row, enabled, with a weight from its
   initial distribution, unless the two are one node, the marking is already
   present (enabled or not), no row is free, or (feedforward genomes) the
   destination already reaches the source through valid connections.
5. Delete connection (conn_delete): a valid connection row is made empty.
6. Attributes of every valid non-input node row and every valid connection
   row (new rows included): a float attribute v with draw u and normal z
   becomes v + power * z when u < mutate_rate, init_mean + init_std * z when
   mutate_rate <= u < mutate_rate + replace_rate, and stays otherwise; an
   activation (aggregation) is replaced, when its draw is below
   replace_rate, by the option of index floor(u2 * n_options), the options in
   ascending code order.

Readings (the paper names the operations and their hyperparameters, not
these details): the order of steps, the split's weights, which parent's genes
are kept, a single try for each structural mutation, no clamping of
attribute values, input rows not mutated. "Picked" means: the candidate rows
in ascending row order, index floor(u * n) of them (the last one for
u * n >= n).

Random numbers are inputs, so that a GPU implementation given the same draws
must reach the same child bit for bit. Per child, uniforms U and normals Z:

  U[0..15]   add node: decision, pick; delete node: decision, pick; add
             connection: decision, source pick, destination pick; delete
             connection: decision, pick; 9..15 unused
  U[16 + r]                    crossover coin of node row r
  U[16 + N_max + r]            crossover coin of connection row r
  U[16 + N_max + C_max + 6 r + k]   node row r attribute draws: k = 0 bias,
             1 response, 2 activation decision, 3 activation pick,
             4 aggregation decision, 5 aggregation pick
  U[16 + 7 N_max + C_max + r]  connection row r weight draw
  Z[0..3]    new node bias, new node response, new connection weight, unused
  Z[4 + 2 r + k]               node row r: k = 0 bias, 1 response
  Z[4 + 2 N_max + r]           connection row r weight

Float attribute updates are two float32 roundings, as written: power * z
rounded, then added to v and rounded (init_mean + init_std * z the same way).

Innovation table of one call: every distinct split marking (a, b) among the
children's node additions gets key next_key + its rank among those markings
in lexicographic order; the same split in two children gives one key (NEAT's
reuse of an innovation within a generation). next_key must exceed every key
in the parents.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Sequence, Tuple

import numpy as np

N_STRUCT = 16
N_Z_HEAD = 4


@dataclasses.dataclass
class MutationParams:
    """Appendix A's hyperparameters, defaults as in Appendix C (feedforward,
    tanh, sum)."""
    node_add: float = 0.2
    node_delete: float = 0.0
    conn_add: float = 0.4
    conn_delete: float = 0.0
    bias_init_mean: float = 0.0
    bias_init_std: float = 1.0
    bias_mutate_power: float = 0.5
    bias_mutate_rate: float = 0.7
    bias_replace_rate: float = 0.1
    resp_init_mean: float = 1.0
    resp_init_std: float = 0.0
    resp_mutate_power: float = 0.0
    resp_mutate_rate: float = 0.0
    resp_replace_rate: float = 0.0
    weight_init_mean: float = 0.0
    weight_init_std: float = 1.0
    weight_mutate_power: float = 0.5
    weight_mutate_rate: float = 0.8
    weight_replace_rate: float = 0.1
    act_default: int = 2
    agg_default: int = 0
    act_replace_rate: float = 0.0
    agg_replace_rate: float = 0.0
    act_options: Tuple[int, ...] = (2,)
    agg_options: Tuple[int, ...] = (0,)
    allow_cycles: bool = False


def n_uniform(N_max: int, C_max: int) -> int:
    return N_STRUCT + 7 * N_max + 2 * C_max


def n_normal(N_max: int, C_max: int) -> int:
    return N_Z_HEAD + 2 * N_max + C_max


f32 = np.float32


def _pick(u, n: int) -> int:
    """Index floor(u * n), at most n - 1 (u * n in float32, as the draws are)."""
    return min(int(np.floor(f32(u) * f32(n))), n - 1)


def _mut_float(v, u, z, mean, std, power, rate, replace):
    """Float attribute rule (two float32 roundings per update)."""
    v, u, z = f32(v), f32(u), f32(z)
    rate, replace = f32(rate), f32(replace)
    if u < rate:
        return f32(v + f32(f32(power) * z))
    if u < f32(rate + replace):
        return f32(f32(mean) + f32(f32(std) * z))
    return v


@dataclasses.dataclass
class Rows:
    """One genome's padded rows (copies, float32 / int32 / uint8 as stored)."""
    key: np.ndarray
    bias: np.ndarray
    resp: np.ndarray
    act: np.ndarray
    agg: np.ndarray
    cin: np.ndarray
    cout: np.ndarray
    w: np.ndarray
    en: np.ndarray

    @classmethod
    def of(cls, pop, g: int) -> "Rows":
        return cls(pop.node_key[g].copy(), pop.node_bias[g].copy(), pop.node_resp[g].copy(),
                   pop.node_act[g].copy(), pop.node_agg[g].copy(), pop.conn_in[g].copy(),
                   pop.conn_out[g].copy(), pop.conn_w[g].copy(), pop.conn_en[g].copy())

    def valid_nodes(self) -> List[int]:
        return [r for r in range(self.key.shape[0]) if self.key[r] >= 0]

    def valid_conns(self) -> List[int]:
        return [r for r in range(self.cin.shape[0]) if self.cin[r] >= 0 and self.cout[r] >= 0]

    def first_empty_node(self) -> int:
        for r in range(self.key.shape[0]):
            if self.key[r] < 0:
                return r
        return -1

    def empty_conns(self) -> List[int]:
        return [r for r in range(self.cin.shape[0]) if not (self.cin[r] >= 0 and self.cout[r] >= 0)]

    def clear_node(self, r: int) -> None:
        self.key[r], self.bias[r], self.resp[r], self.act[r], self.agg[r] = -1, 0, 0, 0, 0

    def clear_conn(self, r: int) -> None:
        self.cin[r], self.cout[r], self.w[r], self.en[r] = -1, -1, 0, 0


def crossover(p1: Rows, p2: Rows, U: np.ndarray) -> Rows:
    """Step 1: the child of fitter parent p1 and parent p2."""
    N, C = p1.key.shape[0], p1.cin.shape[0]
    child = dataclasses.replace(p1, **{f.name: getattr(p1, f.name).copy()
                                       for f in dataclasses.fields(p1)})
    node_of: Dict[int, int] = {}
    for r in p2.valid_nodes():
        node_of.setdefault(int(p2.key[r]), r)
    conn_of: Dict[Tuple[int, int], int] = {}
    for r in p2.valid_conns():
        conn_of.setdefault((int(p2.cin[r]), int(p2.cout[r])), r)
    for r in p1.valid_nodes():
        q = node_of.get(int(p1.key[r]))
        if q is not None and f32(U[N_STRUCT + r]) < f32(0.5):
            child.bias[r], child.resp[r] = p2.bias[q], p2.resp[q]
            child.act[r], child.agg[r] = p2.act[q], p2.agg[q]
    for r in p1.valid_conns():
        q = conn_of.get((int(p1.cin[r]), int(p1.cout[r])))
        if q is not None and f32(U[N_STRUCT + N + r]) < f32(0.5):
            child.w[r], child.en[r] = p2.w[q], p2.en[q]
    return child


def split_choice(child: Rows, U: np.ndarray, prm: MutationParams):
    """Step 2's decision: the connection row to split, or None."""
    if not f32(U[0]) < f32(prm.node_add):
        return None
    cand = [r for r in child.valid_conns() if child.en[r]]
    if not cand:
        return None
    if child.first_empty_node() < 0 or len(child.empty_conns()) < 2:
        return None
    return cand[_pick(U[1], len(cand))]


def innovation_keys(markings: Sequence[Tuple[int, int]], next_key: int):
    """Key of each distinct split marking: next_key + rank in lexicographic order;
    returns (dict marking -> key, the next unused key)."""
    distinct = sorted(set(markings))
    return {m: next_key + i for i, m in enumerate(distinct)}, next_key + len(distinct)


def _reaches(child: Rows, src_key: int, dst_key: int) -> bool:
    """True if a path src_key ->* dst_key exists over valid connection rows."""
    out: Dict[int, List[int]] = {}
    for r in child.valid_conns():
        out.setdefault(int(child.cin[r]), []).append(int(child.cout[r]))
    seen, stack = {src_key}, [src_key]
    while stack:
        k = stack.pop()
        if k == dst_key:
            return True
        for n in out.get(k, []):
            if n not in seen:
                seen.add(n)
                stack.append(n)
    return False


def mutate(child: Rows, U: np.ndarray, Z: np.ndarray, prm: MutationParams, n_in: int,
           n_out: int, split_row, split_key) -> Rows:
    """Steps 2-6 on a crossed-over child (in place; also returned)."""
    N, C = child.key.shape[0], child.cin.shape[0]
    # 2. add node
    if split_row is not None:
        a, b = int(child.cin[split_row]), int(child.cout[split_row])
        w_old = child.w[split_row]
        child.en[split_row] = 0
        rn = child.first_empty_node()
        child.key[rn] = split_key
        child.bias[rn] = f32(f32(prm.bias_init_mean) + f32(f32(prm.bias_init_std) * f32(Z[0])))
        child.resp[rn] = f32(f32(prm.resp_init_mean) + f32(f32(prm.resp_init_std) * f32(Z[1])))
        child.act[rn], child.agg[rn] = prm.act_default, prm.agg_default
        r1, r2 = child.empty_conns()[:2]
        child.cin[r1], child.cout[r1], child.w[r1], child.en[r1] = a, split_key, f32(1.0), 1
        child.cin[r2], child.cout[r2], child.w[r2], child.en[r2] = split_key, b, w_old, 1
    # 3. delete node
    if f32(U[2]) < f32(prm.node_delete):
        cand = [r for r in child.valid_nodes() if child.key[r] >= n_in + n_out]
        if cand:
            r = cand[_pick(U[3], len(cand))]
            k = int(child.key[r])
            child.clear_node(r)
            for c in child.valid_conns():
                if child.cin[c] == k or child.cout[c] == k:
                    child.clear_conn(c)
    # 4. add connection
    if f32(U[4]) < f32(prm.conn_add):
        srcs = [r for r in child.valid_nodes()
                if not (n_in <= child.key[r] < n_in + n_out)]
        dsts = [r for r in child.valid_nodes() if not (0 <= child.key[r] < n_in)]
        free = child.empty_conns()
        if srcs and dsts and free:
            s = int(child.key[srcs[_pick(U[5], len(srcs))]])
            d = int(child.key[dsts[_pick(U[6], len(dsts))]])
            present = any(child.cin[r] == s and child.cout[r] == d for r in child.valid_conns())
            cyc = (not prm.allow_cycles) and _reaches(child, d, s)
            if s != d and not present and not cyc:
                r = free[0]
                child.cin[r], child.cout[r], child.en[r] = s, d, 1
                child.w[r] = f32(f32(prm.weight_init_mean) +
                                 f32(f32(prm.weight_init_std) * f32(Z[2])))
    # 5. delete connection
    if f32(U[7]) < f32(prm.conn_delete):
        cand = child.valid_conns()
        if cand:
            child.clear_conn(cand[_pick(U[8], len(cand))])
    # 6. attributes
    un = N_STRUCT + N + C
    uc = N_STRUCT + 7 * N + C
    for r in child.valid_nodes():
        if child.key[r] < n_in:
            continue
        d = U[un + 6 * r: un + 6 * r + 6]
        child.bias[r] = _mut_float(child.bias[r], d[0], Z[N_Z_HEAD + 2 * r], prm.bias_init_mean,
                                   prm.bias_init_std, prm.bias_mutate_power,
                                   prm.bias_mutate_rate, prm.bias_replace_rate)
        child.resp[r] = _mut_float(child.resp[r], d[1], Z[N_Z_HEAD + 2 * r + 1],
                                   prm.resp_init_mean, prm.resp_init_std, prm.resp_mutate_power,
                                   prm.resp_mutate_rate, prm.resp_replace_rate)
        if f32(d[2]) < f32(prm.act_replace_rate):
            opts = sorted(prm.act_options)
            child.act[r] = opts[_pick(d[3], len(opts))]
        if f32(d[4]) < f32(prm.agg_replace_rate):
            opts = sorted(prm.agg_options)
            child.agg[r] = opts[_pick(d[5], len(opts))]
    for r in child.valid_conns():
        child.w[r] = _mut_float(child.w[r], U[uc + r], Z[N_Z_HEAD + 2 * N + r],
                                prm.weight_init_mean, prm.weight_init_std,
                                prm.weight_mutate_power, prm.weight_mutate_rate,
                                prm.weight_replace_rate)
    return child


def reproduce(pop, parents: np.ndarray, U: np.ndarray, Z: np.ndarray, prm: MutationParams,
              next_key: int):
    """Children of a padded population: parents [n][2] (fitter parent first; a
    negative second parent copies the first unchanged, an elite), uniforms
    U [n][n_uniform], normals Z [n][n_normal]. Returns (arrays dict of the
    children's padded rows, the next unused key)."""
    n = parents.shape[0]
    kids: List[Rows] = []
    splits = []
    for c in range(n):
        p1, p2 = int(parents[c, 0]), int(parents[c, 1])
        r1 = Rows.of(pop, p1)
        if p2 < 0:
            kids.append(r1)
            splits.append(None)
            continue
        child = crossover(r1, Rows.of(pop, p2), U[c])
        kids.append(child)
        sr = split_choice(child, U[c], prm)
        splits.append(None if sr is None else (sr, (int(child.cin[sr]), int(child.cout[sr]))))
    keys, nxt = innovation_keys([s[1] for s in splits if s is not None], next_key)
    for c in range(n):
        if int(parents[c, 1]) < 0:
            continue
        s = splits[c]
        mutate(kids[c], U[c], Z[c], prm, pop.n_in, pop.n_out,
               None if s is None else s[0], None if s is None else keys[s[1]])
    out = {
        "node_key": np.stack([k.key for k in kids]), "node_bias": np.stack([k.bias for k in kids]),
        "node_resp": np.stack([k.resp for k in kids]), "node_act": np.stack([k.act for k in kids]),
        "node_agg": np.stack([k.agg for k in kids]), "conn_in": np.stack([k.cin for k in kids]),
        "conn_out": np.stack([k.cout for k in kids]), "conn_w": np.stack([k.w for k in kids]),
        "conn_en": np.stack([k.en for k in kids]),
    }
    return out, nxt
