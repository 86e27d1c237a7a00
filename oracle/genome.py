"""Decoding and the feedforward transformation (TensorNEAT Sections 3.1 and 3.3).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Readings taken where the paper is silent or garbled:

* A padding row (the paper's NaN row of N-hat / C-hat) is a node row whose key
  is negative, or a connection row whose in- or out-key is negative. Such rows
  may sit anywhere (node removal writes NaN into a row in place, Section 3.2).
* Connection endpoints are historical markers (node keys), not row indices:
  they are looked up among the genome's node keys.
* Only enabled connections enter the expanded connections (the C_exp rule of
  Section 3.3 writes NaN for e = 0); the enabled flag is the third column and
  the attributes start at the fourth.
* The topological order is the level-synchronous one: round r emits, in
  ascending node-row order, every not-yet-emitted node all of whose enabled
  in-edges come from nodes emitted in earlier rounds; r is the node's level.
* The per-node in-edge list (the CSR form of C_exp[:][k]) is ordered by
  ascending connection row.
* Genomes that break the feedforward assumption or the key conventions are
  flagged per genome instead of failing the call: CYCLE (a cycle among enabled
  edges), DANGLING (an enabled edge names a key that no node row holds),
  DUP_CONN (two valid connection rows with the same (in, out) keys, enabled or
  not), DUP_NODE (two node rows with one key), INPUT_DST (an enabled edge ends
  at an input key), MISSING_IO (an input or output key has no node row),
  OVERSIZE (a ragged genome has more rows than the capacity it was declared
  with; it is reported alone, since such a genome is not read further),
  BAD_ATTR (a node row holds an activation or aggregation code outside the
  defined sets). CYCLE is only looked for when no other bit is set (the sort
  needs a well-formed graph).
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Optional, Tuple

import numpy as np

CYCLE = 1
DANGLING = 2
DUP_CONN = 4
DUP_NODE = 8
INPUT_DST = 16
MISSING_IO = 32
OVERSIZE = 64
BAD_ATTR = 128

# Attribute encodings of the library's input format.
ACT_NAMES = {0: "identity", 1: "sigmoid", 2: "tanh", 3: "relu", 4: "sin",
             5: "gaussian", 6: "abs"}
AGG_NAMES = {0: "sum", 1: "product", 2: "max", 3: "min", 4: "mean", 5: "maxabs"}


@dataclasses.dataclass
class Node:
    row: int
    key: int
    bias: float
    resp: float
    act: str
    agg: str


@dataclasses.dataclass
class Conn:
    row: int
    kin: int
    kout: int
    w: float
    enabled: bool


@dataclasses.dataclass
class Genome:
    n_in: int
    n_out: int
    nodes: Dict[int, Node]          # key -> node (first row holding the key)
    conns: List[Conn]               # valid connection rows, ascending row
    status: int = 0


@dataclasses.dataclass
class Transformed:
    status: int
    order: List[int]                      # node keys in topological order
    level: Dict[int, int]                 # key -> level
    in_edges: Dict[int, List[Conn]]       # key -> enabled in-edges, ascending row


def _rows(pop, g):
    if getattr(pop, "node_off", None) is not None:
        ns = slice(int(pop.node_off[g]), int(pop.node_off[g + 1]))
        cs = slice(int(pop.conn_off[g]), int(pop.conn_off[g + 1]))
        return ((pop.node_key[ns], pop.node_bias[ns], pop.node_resp[ns],
                 pop.node_act[ns], pop.node_agg[ns]),
                (pop.conn_in[cs], pop.conn_out[cs], pop.conn_w[cs], pop.conn_en[cs]))
    return ((pop.node_key[g], pop.node_bias[g], pop.node_resp[g], pop.node_act[g],
             pop.node_agg[g]),
            (pop.conn_in[g], pop.conn_out[g], pop.conn_w[g], pop.conn_en[g]))


def decode(pop, g: int) -> Genome:
    """Read genome g's valid rows into dictionaries (Section 3.1)."""
    (key, bias, resp, act, agg), (cin, cout, w, en) = _rows(pop, g)
    status = 0
    if getattr(pop, "node_off", None) is not None:
        if key.shape[0] > pop.N_max or cin.shape[0] > pop.C_max:
            return Genome(int(pop.n_in), int(pop.n_out), {}, [], OVERSIZE)
    nodes: Dict[int, Node] = {}
    for r in range(key.shape[0]):
        k = int(key[r])
        if k < 0:
            continue
        if int(act[r]) not in ACT_NAMES or int(agg[r]) not in AGG_NAMES:
            status |= BAD_ATTR
        if k in nodes:
            status |= DUP_NODE
            continue
        nodes[k] = Node(r, k, float(bias[r]), float(resp[r]),
                        ACT_NAMES.get(int(act[r]), "identity"),
                        AGG_NAMES.get(int(agg[r]), "sum"))
    conns: List[Conn] = []
    for r in range(cin.shape[0]):
        a, b = int(cin[r]), int(cout[r])
        if a < 0 or b < 0:
            continue
        conns.append(Conn(r, a, b, float(w[r]), bool(en[r])))
    return Genome(int(pop.n_in), int(pop.n_out), nodes, conns, status)


def transform(gen: Genome) -> Transformed:
    """Topological order and per-node enabled in-edges (Section 3.3).

    Returns the status bits; when any bit is set the order and edge lists are
    left empty (the genome's outputs are undefined and reported as NaN).
    """
    status = gen.status
    if status & OVERSIZE:
        return Transformed(status, [], {}, {})
    seen = set()
    for c in gen.conns:
        if (c.kin, c.kout) in seen:
            status |= DUP_CONN
        seen.add((c.kin, c.kout))
    for k in range(gen.n_in + gen.n_out):
        if k not in gen.nodes:
            status |= MISSING_IO
    enabled = [c for c in gen.conns if c.enabled]
    for c in enabled:
        if c.kin not in gen.nodes or c.kout not in gen.nodes:
            status |= DANGLING
        if 0 <= c.kout < gen.n_in:
            status |= INPUT_DST
    if status:
        return Transformed(status, [], {}, {})

    remaining = {k: 0 for k in gen.nodes}
    successors: Dict[int, List[int]] = {k: [] for k in gen.nodes}
    in_edges: Dict[int, List[Conn]] = {k: [] for k in gen.nodes}
    for c in enabled:
        remaining[c.kout] += 1
        successors[c.kin].append(c.kout)
        in_edges[c.kout].append(c)
    for k in in_edges:
        in_edges[k].sort(key=lambda c: c.row)

    order: List[int] = []
    level: Dict[int, int] = {}
    r = 0
    while True:
        ready = [k for k in gen.nodes if remaining[k] == 0 and k not in level]
        if not ready:
            break
        ready.sort(key=lambda k: gen.nodes[k].row)
        for k in ready:
            order.append(k)
            level[k] = r
        for k in ready:
            for s in successors[k]:
                remaining[s] -= 1
        r += 1
    if len(order) < len(gen.nodes):
        return Transformed(status | CYCLE, [], {}, {})
    return Transformed(0, order, level, in_edges)


def transform_population(pop) -> List[Tuple[Genome, Transformed]]:
    return [(g, transform(g)) for g in (decode(pop, i) for i in range(pop.P))]


def transform_arrays(pop, genomes: Optional[List[int]] = None) -> dict:
    """The transformation in the library's array form, for bit-exact comparison.

    Per genome (positions p are topological positions):
      status            - status bits
      n_valid           - number of nodes (valid only when status == 0)
      order[p]          - node row of the node at position p
      level[p]          - its level
      row_ptr[p]        - start of its in-edges in the edge arrays (p = 0..n_valid)
      edge_src[e]       - topological position of the edge's source node
      edge_row[e]       - connection row of the edge
      edge_w[e]         - its weight (float32, copied)
    Each genome's arrays are returned as Python lists in a list over genomes.
    """
    idx = range(pop.P) if genomes is None else genomes
    out = {k: [] for k in ("status", "n_valid", "order", "level", "row_ptr",
                           "edge_src", "edge_row", "edge_w")}
    for g in idx:
        gen = decode(pop, g)
        tr = transform(gen)
        out["status"].append(tr.status)
        if tr.status:
            for k in ("n_valid", "order", "level", "row_ptr", "edge_src",
                      "edge_row", "edge_w"):
                out[k].append(None)
            continue
        pos = {k: p for p, k in enumerate(tr.order)}
        out["n_valid"].append(len(tr.order))
        out["order"].append([gen.nodes[k].row for k in tr.order])
        out["level"].append([tr.level[k] for k in tr.order])
        rp, es, er, ew = [0], [], [], []
        for k in tr.order:
            for c in tr.in_edges[k]:
                es.append(pos[c.kin])
                er.append(c.row)
                ew.append(np.float32(c.w))
            rp.append(len(es))
        out["row_ptr"].append(rp)
        out["edge_src"].append(es)
        out["edge_row"].append(er)
        out["edge_w"].append(ew)
    return out
