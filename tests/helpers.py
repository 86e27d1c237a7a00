"""Small builders shared by the tests (inputs only; no method arithmetic)."""
import json
import os

import numpy as np

import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load_golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def population_from_rows(genomes, n_in, n_out, N_max=None, C_max=None):
    """Padded population from per-genome row lists.

    genomes: list of (nodes, conns); nodes rows [key, bias, resp, act, agg],
    conn rows [in, out, w, enabled]; rows keep their list position.
    """
    N_max = N_max or max(1, max(len(n) for n, _ in genomes))
    C_max = C_max or max(1, max(len(c) for _, c in genomes))
    P = len(genomes)
    pop = synth.Population(
        n_in, n_out, N_max, C_max,
        np.full((P, N_max), -1, np.int32), np.zeros((P, N_max), np.float32),
        np.zeros((P, N_max), np.float32), np.zeros((P, N_max), np.uint8),
        np.zeros((P, N_max), np.uint8),
        np.full((P, C_max), -1, np.int32), np.full((P, C_max), -1, np.int32),
        np.zeros((P, C_max), np.float32), np.zeros((P, C_max), np.uint8))
    for g, (nodes, conns) in enumerate(genomes):
        for r, row in enumerate(nodes):
            if row is None:
                continue
            k, b, rho, a, ag = row
            pop.node_key[g, r] = k
            pop.node_bias[g, r] = b
            pop.node_resp[g, r] = rho
            pop.node_act[g, r] = a
            pop.node_agg[g, r] = ag
        for r, row in enumerate(conns):
            if row is None:
                continue
            i, o, w, e = row
            pop.conn_in[g, r] = i
            pop.conn_out[g, r] = o
            pop.conn_w[g, r] = w
            pop.conn_en[g, r] = e
    return pop


def mlp_genome(rng, sizes, hidden_act=2, out_act=0, resp=None):
    """A layered, fully connected genome I -> H1 -> ... -> O and its dense
    parameters (float32): returns (nodes, conns, weights, biases) where
    weights[l] is [fan_in][fan_out] and biases[l] is [fan_out].
    Keys: inputs 0..I-1, outputs I..I+O-1, hidden from I+O upward."""
    I, O = sizes[0], sizes[-1]
    keys = [list(range(I))]
    nxt = I + O
    for h in sizes[1:-1]:
        keys.append(list(range(nxt, nxt + h)))
        nxt += h
    keys.append(list(range(I, I + O)))
    nodes = [[k, float(rng.standard_normal()), 1.0, 0, 0] for k in keys[0]]
    weights, biases, conns = [], [], []
    for l in range(1, len(keys)):
        W = rng.standard_normal((len(keys[l - 1]), len(keys[l]))).astype(np.float32)
        b = rng.standard_normal(len(keys[l])).astype(np.float32)
        weights.append(W)
        biases.append(b)
        act = out_act if l == len(keys) - 1 else hidden_act
        for j, k in enumerate(keys[l]):
            nodes.append([k, float(b[j]), 1.0 if resp is None else resp, act, 0])
        for i, ki in enumerate(keys[l - 1]):
            for j, kj in enumerate(keys[l]):
                conns.append([ki, kj, float(W[i, j]), 1])
    return nodes, conns, weights, biases
