"""Seeded synthetic NEAT populations in the structure-of-arrays layout.

Layout (the tensorized encoding of the paper, Section 3.1, with the padding
rows of N-hat / C-hat marked by key -1 instead of NaN):

* node rows:  key int32, bias float32, response float32, activation uint8,
  aggregation uint8
* connection rows: in-key int32, out-key int32, weight float32, enabled uint8

Padded populations store genome g's rows at ``[g, 0:N_max]`` / ``[g, 0:C_max]``.
Ragged populations concatenate every genome's rows and add ``node_off`` /
``conn_off`` (int64, length P+1).

Keys follow the genome interface of Appendix B: inputs are keys 0..I-1,
outputs I..I+O-1; hidden keys are larger.

Growth follows NEAT's incremental expansion (Section 2.1): every genome starts
from the minimal fully connected input->output genome and receives seeded
add-node / add-connection mutations in the paper's 0.2 : 0.4 ratio (Appendix C).
A population-wide split table gives the same new key whenever the same
connection is split, so genomes share homologous genes as with NEAT's
historical markers. Acyclicity of added connections is kept with a
population-wide rank per key (inputs 0, outputs 1, a split node halfway between
the ranks of the split connection's endpoints); a connection is only added from
a lower to a strictly higher rank. This is a property of the generator, not of
the method: the transform itself accepts any graph and flags cycles.

Nothing here evaluates a network: only inputs are produced.
"""
from __future__ import annotations

import dataclasses
from typing import Optional, Sequence

import numpy as np

# Input encodings of the activation / aggregation attributes, as declared by the
# library's C header (enum tn_act / tn_agg).
ACT = {"identity": 0, "sigmoid": 1, "tanh": 2, "relu": 3, "sin": 4,
       "gaussian": 5, "abs": 6}
AGG = {"sum": 0, "product": 1, "max": 2, "min": 3, "mean": 4, "maxabs": 5}

# Seeds of the five workloads; observation seeds are these plus 100.
CONFIG_SEEDS = {"xor": 1, "control": 2, "batching": 3, "differentiation": 4,
                "cppn": 5, "recurrent": 6}


@dataclasses.dataclass
class Population:
    n_in: int
    n_out: int
    N_max: int
    C_max: int
    node_key: np.ndarray
    node_bias: np.ndarray
    node_resp: np.ndarray
    node_act: np.ndarray
    node_agg: np.ndarray
    conn_in: np.ndarray
    conn_out: np.ndarray
    conn_w: np.ndarray
    conn_en: np.ndarray
    node_off: Optional[np.ndarray] = None
    conn_off: Optional[np.ndarray] = None

    @property
    def ragged(self) -> bool:
        return self.node_off is not None

    @property
    def P(self) -> int:
        if self.ragged:
            return int(self.node_off.shape[0] - 1)
        return int(self.node_key.shape[0])

    def node_rows(self, g: int) -> dict:
        """Genome g's node rows (views), padding included."""
        if self.ragged:
            s = slice(int(self.node_off[g]), int(self.node_off[g + 1]))
            return {k: getattr(self, "node_" + k)[s] for k in
                    ("key", "bias", "resp", "act", "agg")}
        return {k: getattr(self, "node_" + k)[g] for k in
                ("key", "bias", "resp", "act", "agg")}

    def conn_rows(self, g: int) -> dict:
        """Genome g's connection rows (views), padding included."""
        if self.ragged:
            s = slice(int(self.conn_off[g]), int(self.conn_off[g + 1]))
            return {k: getattr(self, "conn_" + k)[s] for k in
                    ("in", "out", "w", "en")}
        return {k: getattr(self, "conn_" + k)[g] for k in
                ("in", "out", "w", "en")}

    def arrays(self) -> dict:
        d = {f.name: getattr(self, f.name) for f in dataclasses.fields(self)}
        return {k: v for k, v in d.items() if isinstance(v, np.ndarray)}

    def nbytes_valid(self) -> int:
        """Bytes of the non-empty rows (14 B per node row, 13 B per connection row)."""
        nk = self.node_key
        cin, cout = self.conn_in, self.conn_out
        n_nodes = int(np.count_nonzero(nk >= 0))
        n_conns = int(np.count_nonzero((cin >= 0) & (cout >= 0)))
        return 14 * n_nodes + 13 * n_conns


# --------------------------------------------------------------------------
# Genome growth
# --------------------------------------------------------------------------

class _Innovations:
    """Population-wide split table and key ranks."""

    def __init__(self, n_in: int, n_out: int):
        self.next_key = n_in + n_out
        self.split = {}
        self.rank = {}
        for k in range(n_in):
            self.rank[k] = 0.0
        for k in range(n_in, n_in + n_out):
            self.rank[k] = 1.0

    def split_key(self, a: int, b: int) -> int:
        h = self.split.get((a, b))
        if h is None:
            h = self.next_key
            self.next_key += 1
            self.split[(a, b)] = h
            self.rank[h] = 0.5 * (self.rank[a] + self.rank[b])
        return h


def _act_code(rng, choices: Sequence[str]) -> int:
    return ACT[choices[int(rng.integers(len(choices)))]]


def grow_population(P: int, n_in: int, n_out: int, N_max: int, C_max: int,
                    n_mutations, rng: np.random.Generator, *,
                    hidden_acts: Sequence[str], output_acts: Sequence[str],
                    hidden_cap: Optional[int] = None,
                    conn_cap: Optional[int] = None,
                    disable_p: float = 0.0) -> Population:
    """Grow P genomes from the minimal fully connected genome.

    ``n_mutations`` is an int or an array of P ints. Each mutation is an
    add-node with probability 1/3, else an add-connection (20 tries).
    """
    if np.isscalar(n_mutations):
        n_mutations = np.full(P, int(n_mutations), dtype=np.int64)
    hidden_cap = N_max - n_in - n_out if hidden_cap is None else hidden_cap
    conn_cap = C_max if conn_cap is None else conn_cap
    inn = _Innovations(n_in, n_out)
    node_key = np.full((P, N_max), -1, np.int32)
    node_bias = np.zeros((P, N_max), np.float32)
    node_resp = np.zeros((P, N_max), np.float32)
    node_act = np.zeros((P, N_max), np.uint8)
    node_agg = np.zeros((P, N_max), np.uint8)
    conn_in = np.full((P, C_max), -1, np.int32)
    conn_out = np.full((P, C_max), -1, np.int32)
    conn_w = np.zeros((P, C_max), np.float32)
    conn_en = np.zeros((P, C_max), np.uint8)

    for g in range(P):
        # nodes: list of [key, bias, resp, act, agg]
        nodes = []
        for k in range(n_in):
            nodes.append([k, rng.standard_normal(), 1.0, ACT["identity"], AGG["sum"]])
        for k in range(n_in, n_in + n_out):
            nodes.append([k, rng.standard_normal(), 1.0, _act_code(rng, output_acts),
                          AGG["sum"]])
        conns = []   # [in, out, w, en]
        present = set()
        for i in range(n_in):
            for o in range(n_in, n_in + n_out):
                conns.append([i, o, rng.standard_normal(), 1])
                present.add((i, o))
        keys_here = set(range(n_in + n_out))
        hidden_here = []
        for _ in range(int(n_mutations[g])):
            if rng.random() < 1.0 / 3.0:
                enabled = [c for c in conns if c[3] == 1]
                if not enabled:
                    continue
                c = enabled[int(rng.integers(len(enabled)))]
                if len(hidden_here) >= hidden_cap or len(conns) + 2 > conn_cap:
                    continue
                h = inn.split_key(c[0], c[1])
                if h in keys_here:
                    continue
                c[3] = 0
                nodes.append([h, rng.standard_normal(), 1.0,
                              _act_code(rng, hidden_acts), AGG["sum"]])
                keys_here.add(h)
                hidden_here.append(h)
                conns.append([c[0], h, rng.standard_normal(), 1])
                conns.append([h, c[1], rng.standard_normal(), 1])
                present.add((c[0], h))
                present.add((h, c[1]))
            else:
                if len(conns) >= conn_cap:
                    continue
                srcs = list(range(n_in)) + hidden_here
                dsts = hidden_here + list(range(n_in, n_in + n_out))
                for _try in range(20):
                    s = srcs[int(rng.integers(len(srcs)))]
                    d = dsts[int(rng.integers(len(dsts)))]
                    if (s, d) in present or not inn.rank[s] < inn.rank[d]:
                        continue
                    conns.append([s, d, rng.standard_normal(), 1])
                    present.add((s, d))
                    break
        if disable_p > 0.0:
            for c in conns:
                if rng.random() < disable_p:
                    c[3] = 0
        for r, n in enumerate(nodes):
            node_key[g, r] = n[0]
            node_bias[g, r] = n[1]
            node_resp[g, r] = n[2]
            node_act[g, r] = n[3]
            node_agg[g, r] = n[4]
        for r, c in enumerate(conns):
            conn_in[g, r] = c[0]
            conn_out[g, r] = c[1]
            conn_w[g, r] = c[2]
            conn_en[g, r] = c[3]
    return Population(n_in, n_out, N_max, C_max, node_key, node_bias, node_resp,
                      node_act, node_agg, conn_in, conn_out, conn_w, conn_en)


def random_dag_population(P: int, n_in: int, n_out: int, rng: np.random.Generator,
                          *, h_lo: int = 10, h_hi: int = 500, c_lo: float = 2.0,
                          c_hi: float = 4.0, c_cap: int = 2000,
                          disable_p: float = 0.15,
                          acts: Sequence[str] = ("tanh", "sigmoid", "relu", "identity")
                          ) -> Population:
    """Ragged population of independent random DAGs of very uneven size.

    Hidden count H = round(exp(U(ln h_lo, ln h_hi))); connection count
    min(c_cap, round(U(c_lo, c_hi) * H)). Each hidden node gets a random rank;
    a connection goes from an input or hidden node to a hidden or output node of
    strictly higher rank (inputs lowest, outputs highest).
    """
    node_blocks, conn_blocks = [], []
    n_counts, c_counts = [], []
    act_codes = np.array([ACT[a] for a in acts], np.uint8)
    for g in range(P):
        H = int(round(float(np.exp(rng.uniform(np.log(h_lo), np.log(h_hi))))))
        C = int(min(c_cap, round(rng.uniform(c_lo, c_hi) * H)))
        N = n_in + n_out + H
        keys = np.arange(N, dtype=np.int32)
        bias = rng.standard_normal(N).astype(np.float32)
        resp = np.ones(N, np.float32)
        act = np.zeros(N, np.uint8)
        act[n_in:] = act_codes[rng.integers(len(act_codes), size=N - n_in)]
        agg = np.zeros(N, np.uint8)
        # ranks: inputs -1, hidden permutation 0..H-1, outputs H
        rank = np.empty(N, np.int64)
        rank[:n_in] = -1
        rank[n_in:n_in + n_out] = H
        rank[n_in + n_out:] = rng.permutation(H)
        srcs = np.concatenate([np.arange(n_in), np.arange(n_in + n_out, N)])
        dsts = np.arange(n_in, N)
        chosen_s = np.empty(0, np.int64)
        chosen_d = np.empty(0, np.int64)
        seen = set()
        while chosen_s.shape[0] < C:
            m = 3 * (C - chosen_s.shape[0]) + 16
            s = srcs[rng.integers(len(srcs), size=m)]
            d = dsts[rng.integers(len(dsts), size=m)]
            ok = rank[s] < rank[d]
            s, d = s[ok], d[ok]
            add_s, add_d = [], []
            for a, b in zip(s.tolist(), d.tolist()):
                if (a, b) in seen:
                    continue
                seen.add((a, b))
                add_s.append(a)
                add_d.append(b)
                if chosen_s.shape[0] + len(add_s) >= C:
                    break
            chosen_s = np.concatenate([chosen_s, np.array(add_s, np.int64)])
            chosen_d = np.concatenate([chosen_d, np.array(add_d, np.int64)])
        w = rng.standard_normal(C).astype(np.float32)
        en = (rng.random(C) >= disable_p).astype(np.uint8)
        node_blocks.append((keys, bias, resp, act, agg))
        conn_blocks.append((chosen_s.astype(np.int32), chosen_d.astype(np.int32), w, en))
        n_counts.append(N)
        c_counts.append(C)
    node_off = np.zeros(P + 1, np.int64)
    node_off[1:] = np.cumsum(n_counts)
    conn_off = np.zeros(P + 1, np.int64)
    conn_off[1:] = np.cumsum(c_counts)
    cat = lambda blocks, i: np.concatenate([b[i] for b in blocks])
    return Population(n_in, n_out, int(max(n_counts)), int(max(c_counts)),
                      cat(node_blocks, 0), cat(node_blocks, 1), cat(node_blocks, 2),
                      cat(node_blocks, 3), cat(node_blocks, 4),
                      cat(conn_blocks, 0), cat(conn_blocks, 1), cat(conn_blocks, 2),
                      cat(conn_blocks, 3), node_off, conn_off)


# --------------------------------------------------------------------------
# The five workloads
# --------------------------------------------------------------------------

def xor_population(seed: int = CONFIG_SEEDS["xor"], P: int = 150) -> Population:
    """XOR-sized: 3 inputs (2 + bias), 1 output, 0-20 mutations, N_max 16, C_max 32."""
    rng = np.random.default_rng(seed)
    muts = rng.integers(0, 21, size=P)
    return grow_population(P, 3, 1, 16, 32, muts, rng, hidden_acts=("sigmoid",),
                           output_acts=("sigmoid",), hidden_cap=10, conn_cap=30)


def control_population(seed: int = CONFIG_SEEDS["control"], P: int = 1000) -> Population:
    """Control-policy sized: 17 -> 6, 50 mutations, 15% disabled, N_max 64, C_max 256."""
    rng = np.random.default_rng(seed)
    acts = ("tanh", "sigmoid", "relu", "identity")
    return grow_population(P, 17, 6, 64, 256, 50, rng, hidden_acts=acts,
                           output_acts=acts, disable_p=0.15)


def batching_population(seed: int = CONFIG_SEEDS["batching"], P: int = 10000) -> Population:
    """Uneven sizes: 27 -> 8, hidden log-uniform in [10, 500], 2-4x connections (<= 2000)."""
    rng = np.random.default_rng(seed)
    return random_dag_population(P, 27, 8, rng)


def differentiation_population(seed: int = CONFIG_SEEDS["differentiation"],
                               P: int = 4096) -> Population:
    """4 -> 2, 50 mutations, 15% disabled, tanh hidden, identity outputs, N_max 64, C_max 256."""
    rng = np.random.default_rng(seed)
    return grow_population(P, 4, 2, 64, 256, 50, rng, hidden_acts=("tanh",),
                           output_acts=("identity",), disable_p=0.15)


def cppn_population(seed: int = CONFIG_SEEDS["cppn"], P: int = 1000) -> Population:
    """CPPN genomes: 5 inputs (x_s, y_s, x_t, y_t, bias) -> 1 tanh output, 30 mutations,
    hidden activations from {sin, gaussian, tanh, abs}, N_max 32, C_max 96."""
    rng = np.random.default_rng(seed)
    return grow_population(P, 5, 1, 32, 96, 30, rng,
                           hidden_acts=("sin", "gaussian", "tanh", "abs"),
                           output_acts=("tanh",))


def recurrent_population(seed: int = CONFIG_SEEDS["recurrent"], P: int = 1000, back_edges: int = 12) -> Population:
    """Recurrent-network sized: the control population's genomes (17 -> 6, N_max
    64, C_max 256) plus up to ``back_edges`` extra enabled connections per
    genome whose destination is a hidden node, an output or the source itself
    (self-loops and edges against the growth order, so most genomes gain
    cycles); weights N(0, 1) scaled by 0.5, markings kept unique."""
    pop = control_population(P=P)
    rng = np.random.default_rng(seed)
    for g in range(P):
        keys = pop.node_key[g][pop.node_key[g] >= 0]
        srcs = keys[(keys < pop.n_in) | (keys >= pop.n_in + pop.n_out)]
        srcs = np.concatenate([srcs, keys[(keys >= pop.n_in) & (keys < pop.n_in + pop.n_out)]])
        dsts = keys[keys >= pop.n_in]
        valid = (pop.conn_in[g] >= 0) & (pop.conn_out[g] >= 0)
        present = set(zip(pop.conn_in[g][valid].tolist(), pop.conn_out[g][valid].tolist()))
        free = list(np.flatnonzero(~valid))
        for _ in range(back_edges):
            if not free:
                break
            d = int(rng.choice(dsts))
            a = d if rng.random() < 0.25 else int(rng.choice(srcs))
            if (a, d) in present:
                continue
            r = free.pop(0)
            pop.conn_in[g, r], pop.conn_out[g, r] = a, d
            pop.conn_w[g, r] = np.float32(0.5 * rng.standard_normal())
            pop.conn_en[g, r] = 1
            present.add((a, d))
    return pop


# --------------------------------------------------------------------------
# Observations and targets
# --------------------------------------------------------------------------

def xor_inputs() -> np.ndarray:
    """The four XOR rows; the third input is the bias input fixed at 1.0."""
    return np.array([[0, 0, 1], [0, 1, 1], [1, 0, 1], [1, 1, 1]], np.float32)


def xor_targets() -> np.ndarray:
    return np.array([[0], [1], [1], [0]], np.float32)


def normal_obs(P: int, B: int, I: int, seed: int) -> np.ndarray:
    """Per-genome N(0,1) observations, float32 [P][B][I]."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((P, B, I), dtype=np.float32)


def uniform_inputs(B: int, I: int, seed: int) -> np.ndarray:
    """Shared U(-1,1) inputs, float32 [B][I]."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, size=(B, I)).astype(np.float32)


def target_mlp(X: np.ndarray, hidden: int, n_out: int, seed: int) -> np.ndarray:
    """Regression targets from a fixed seeded MLP: tanh hidden layer (weights
    N(0,1)/sqrt(fan_in), zero biases) and a linear output layer. float32 [B][O]."""
    rng = np.random.default_rng(seed)
    I = X.shape[1]
    W1 = rng.standard_normal((I, hidden)) / np.sqrt(I)
    W2 = rng.standard_normal((hidden, n_out)) / np.sqrt(hidden)
    return (np.tanh(X.astype(np.float64) @ W1) @ W2).astype(np.float32)


# --------------------------------------------------------------------------
# Layout transformations used to build test cases
# --------------------------------------------------------------------------

def _copy(pop: Population) -> Population:
    return dataclasses.replace(pop, **{k: v.copy() for k, v in pop.arrays().items()})


def permute_rows(pop: Population, rng: np.random.Generator, nodes: bool = True,
                 conns: bool = True) -> Population:
    """Shuffle each padded genome's node rows and/or connection rows (padding too)."""
    assert not pop.ragged
    out = _copy(pop)
    for g in range(pop.P):
        if nodes:
            p = rng.permutation(pop.N_max)
            for k in ("key", "bias", "resp", "act", "agg"):
                getattr(out, "node_" + k)[g] = getattr(pop, "node_" + k)[g][p]
        if conns:
            p = rng.permutation(pop.C_max)
            for k in ("in", "out", "w", "en"):
                getattr(out, "conn_" + k)[g] = getattr(pop, "conn_" + k)[g][p]
    return out


def insert_holes(pop: Population, rng: np.random.Generator) -> Population:
    """Move each padded genome's valid rows apart so that empty rows sit between them
    (row order among valid rows is kept)."""
    assert not pop.ragged
    out = _copy(pop)
    for g in range(pop.P):
        for prefix, cap, names, valid in (
                ("node_", pop.N_max, ("key", "bias", "resp", "act", "agg"),
                 pop.node_key[g] >= 0),
                ("conn_", pop.C_max, ("in", "out", "w", "en"),
                 (pop.conn_in[g] >= 0) & (pop.conn_out[g] >= 0))):
            idx = np.flatnonzero(valid)
            n = idx.shape[0]
            if n == 0 or n == cap:
                continue
            dest = np.sort(rng.choice(cap, size=n, replace=False))
            for k in names:
                src = getattr(pop, prefix + k)[g]
                dst = getattr(out, prefix + k)[g]
                fill = -1 if k in ("key", "in", "out") else 0
                vals = src[idx].copy()
                dst[:] = fill
                dst[dest] = vals
    return out


def to_ragged(pop: Population) -> Population:
    """Drop padding rows: concatenate each genome's valid rows (in row order)."""
    assert not pop.ragged
    nb, cb = [], []
    n_counts, c_counts = [], []
    for g in range(pop.P):
        nv = np.flatnonzero(pop.node_key[g] >= 0)
        cv = np.flatnonzero((pop.conn_in[g] >= 0) & (pop.conn_out[g] >= 0))
        nb.append([getattr(pop, "node_" + k)[g][nv] for k in ("key", "bias", "resp", "act", "agg")])
        cb.append([getattr(pop, "conn_" + k)[g][cv] for k in ("in", "out", "w", "en")])
        n_counts.append(nv.shape[0])
        c_counts.append(cv.shape[0])
    node_off = np.zeros(pop.P + 1, np.int64)
    node_off[1:] = np.cumsum(n_counts)
    conn_off = np.zeros(pop.P + 1, np.int64)
    conn_off[1:] = np.cumsum(c_counts)
    cat = lambda blocks, i, dt: (np.concatenate([b[i] for b in blocks]) if blocks
                                 else np.zeros(0, dt))
    return Population(pop.n_in, pop.n_out, max(1, max(n_counts, default=1)),
                      max(1, max(c_counts, default=1)),
                      cat(nb, 0, np.int32), cat(nb, 1, np.float32), cat(nb, 2, np.float32),
                      cat(nb, 3, np.uint8), cat(nb, 4, np.uint8),
                      cat(cb, 0, np.int32), cat(cb, 1, np.int32), cat(cb, 2, np.float32),
                      cat(cb, 3, np.uint8), node_off, conn_off)


def to_padded(pop: Population, N_max: Optional[int] = None,
              C_max: Optional[int] = None) -> Population:
    """Pad a ragged population to uniform capacity."""
    assert pop.ragged
    N_max = pop.N_max if N_max is None else N_max
    C_max = pop.C_max if C_max is None else C_max
    P = pop.P
    out = Population(pop.n_in, pop.n_out, N_max, C_max,
                     np.full((P, N_max), -1, np.int32), np.zeros((P, N_max), np.float32),
                     np.zeros((P, N_max), np.float32), np.zeros((P, N_max), np.uint8),
                     np.zeros((P, N_max), np.uint8),
                     np.full((P, C_max), -1, np.int32), np.full((P, C_max), -1, np.int32),
                     np.zeros((P, C_max), np.float32), np.zeros((P, C_max), np.uint8))
    for g in range(P):
        nr = pop.node_rows(g)
        cr = pop.conn_rows(g)
        n = nr["key"].shape[0]
        c = cr["in"].shape[0]
        assert n <= N_max and c <= C_max
        for k, v in nr.items():
            getattr(out, "node_" + k)[g, :n] = v
        for k, v in cr.items():
            getattr(out, "conn_" + k)[g, :c] = v
    return out


def subset(pop: Population, genomes: Sequence[int]) -> Population:
    """A population made of the listed genomes (same layout kind)."""
    genomes = [int(g) for g in genomes]
    if not pop.ragged:
        return Population(pop.n_in, pop.n_out, pop.N_max, pop.C_max,
                          *[getattr(pop, n)[genomes].copy() for n in
                            ("node_key", "node_bias", "node_resp", "node_act", "node_agg",
                             "conn_in", "conn_out", "conn_w", "conn_en")])
    if not genomes:
        z = lambda a: a[:0].copy()
        return Population(pop.n_in, pop.n_out, pop.N_max, pop.C_max,
                          *[z(getattr(pop, n)) for n in
                            ("node_key", "node_bias", "node_resp", "node_act", "node_agg",
                             "conn_in", "conn_out", "conn_w", "conn_en")],
                          np.zeros(1, np.int64), np.zeros(1, np.int64))
    nb = [pop.node_rows(g) for g in genomes]
    cb = [pop.conn_rows(g) for g in genomes]
    node_off = np.zeros(len(genomes) + 1, np.int64)
    node_off[1:] = np.cumsum([b["key"].shape[0] for b in nb])
    conn_off = np.zeros(len(genomes) + 1, np.int64)
    conn_off[1:] = np.cumsum([b["in"].shape[0] for b in cb])
    cat = lambda bl, k: np.concatenate([b[k] for b in bl])
    return Population(pop.n_in, pop.n_out,
                      int(max(b["key"].shape[0] for b in nb)),
                      int(max(b["in"].shape[0] for b in cb)),
                      cat(nb, "key"), cat(nb, "bias"), cat(nb, "resp"), cat(nb, "act"),
                      cat(nb, "agg"), cat(cb, "in"), cat(cb, "out"), cat(cb, "w"),
                      cat(cb, "en"), node_off, conn_off)


def to_paper_layout(pop: Population):
    """The population as the paper's float tensors (Section 3.1): P_N [P][N_max][5]
    rows [k, bias, response, act, agg] and P_C [P][C_max][4] rows [k_in, k_out, e, w],
    with every empty row all NaN (padded populations only)."""
    assert not pop.ragged
    P = pop.P
    PN = np.full((P, pop.N_max, 5), np.nan, np.float32)
    PC = np.full((P, pop.C_max, 4), np.nan, np.float32)
    nv = pop.node_key >= 0
    cv = (pop.conn_in >= 0) & (pop.conn_out >= 0)
    for j, a in enumerate((pop.node_key, pop.node_bias, pop.node_resp, pop.node_act,
                           pop.node_agg)):
        PN[..., j] = np.where(nv, a.astype(np.float32), np.float32(np.nan))
    for j, a in enumerate((pop.conn_in, pop.conn_out, pop.conn_en, pop.conn_w)):
        PC[..., j] = np.where(cv, a.astype(np.float32), np.float32(np.nan))
    return PN, PC


def reproduction_draws(n_children: int, n_uniform: int, n_normal: int, seed: int):
    """Random draws consumed by crossover and mutation, as inputs: uniforms in
    [0, 1) [n][n_uniform] and standard normals [n][n_normal], float32."""
    rng = np.random.default_rng(seed)
    U = rng.random((n_children, n_uniform), dtype=np.float32)
    Z = rng.standard_normal((n_children, n_normal), dtype=np.float32)
    return U, Z
