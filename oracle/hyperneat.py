"""HyperNEAT: a CPPN genome queried over a grid substrate, and the substrate
network it encodes (the indirect encoding among TensorNEAT's algorithms,
Section 4.4, after Stanley et al.'s HyperNEAT).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The CPPN is an ordinary genome evaluated by ``inference.forward``; a substrate
connection from node s to node t gets the weight
    w(s, t) = cppn(x_s, y_s, x_t, y_t, 1)
and the substrate is a dense two-layer network with no biases,
    H = tanh(X W1),  Y = H W2.
Readings (the paper fixes no geometry):
* input and hidden layers are n x n grids at (x, y) = (-1 + 2c/(n-1), -1 + 2r/(n-1))
  for node index n*r + c; the m outputs sit at (-1 + 2j/(m-1), 0);
* one CPPN gives both layers' weights (its inputs carry no layer index);
* a weight of magnitude below the threshold (0.2) is 0; the others are kept
  unchanged (no rescaling);
* training signal: a fixed upstream gradient dY, i.e. L = sum(dY * Y); the
  CPPN's parameters receive dL/dw(s, t) only through weights that survived
  the threshold (the threshold's derivative is 0 elsewhere).
A parity-tested GPU path that rounds weights and inputs to bfloat16 is
compared against these float64 values with a tolerance derived from that
rounding (``error_scale``).
"""
from __future__ import annotations

from typing import Dict, Tuple

import numpy as np

from .adjoint import backward
from .inference import forward

THRESHOLD = 0.2


def grid_coords(n: int) -> np.ndarray:
    """[n*n][2] coordinates of an n x n grid layer, node index n*r + c."""
    r, c = np.divmod(np.arange(n * n), n)
    step = 2.0 / (n - 1)
    return np.stack([-1.0 + step * c, -1.0 + step * r], axis=1)


def row_coords(m: int) -> np.ndarray:
    """[m][2] coordinates of m nodes on the line y = 0."""
    x = -1.0 + 2.0 * np.arange(m) / (m - 1) if m > 1 else np.zeros(1)
    return np.stack([x, np.zeros(m)], axis=1)


def query_inputs(src: np.ndarray, dst: np.ndarray) -> np.ndarray:
    """CPPN inputs [S*T][5] for every (source s, target t), s-major."""
    S, T = len(src), len(dst)
    q = np.empty((S * T, 5))
    q[:, 0] = np.repeat(src[:, 0], T)
    q[:, 1] = np.repeat(src[:, 1], T)
    q[:, 2] = np.tile(dst[:, 0], S)
    q[:, 3] = np.tile(dst[:, 1], S)
    q[:, 4] = 1.0
    return q


def cppn_weights(gen, tr, src: np.ndarray, dst: np.ndarray) -> np.ndarray:
    """Raw CPPN outputs [S][T] (before the threshold)."""
    y = forward(gen, tr, query_inputs(src, dst))
    return y[:, 0].reshape(len(src), len(dst))


def threshold(w: np.ndarray, thr: float = THRESHOLD) -> np.ndarray:
    return np.where(np.abs(w) < thr, 0.0, w)


def substrate_forward(X: np.ndarray, W1: np.ndarray, W2: np.ndarray):
    """(H, Y) for inputs X [B][S1]: H = tanh(X W1), Y = H W2."""
    H = np.tanh(np.asarray(X, np.float64) @ W1)
    return H, H @ W2


def substrate_backward(X: np.ndarray, W2: np.ndarray, H: np.ndarray, dY: np.ndarray):
    """(dW1, dW2) of L = sum(dY * Y):
    dW2 = H^T dY;  dZ = (dY W2^T) * (1 - H^2);  dW1 = X^T dZ."""
    X = np.asarray(X, np.float64)
    dY = np.asarray(dY, np.float64)
    dW2 = H.T @ dY
    dZ = (dY @ W2.T) * (1.0 - H * H)
    return X.T @ dZ, dW2


def cppn_gradient(gen, tr, src: np.ndarray, dst: np.ndarray, raw: np.ndarray,
                  dW: np.ndarray, thr: float = THRESHOLD):
    """(dW_cppn, db_cppn) dicts row -> value: the CPPN adjoint with upstream
    gradient dW [S][T] at every query, zero where the weight was thresholded."""
    up = np.where(np.abs(raw) < thr, 0.0, dW).reshape(-1, 1)
    return backward(gen, tr, query_inputs(src, dst), up)


def error_scale(X: np.ndarray, W1: np.ndarray, W2: np.ndarray, H: np.ndarray) -> np.ndarray:
    """First-order scale [B][m] of |Y| under relative perturbations of every
    factor of the two products: sum_k |W2[k]| (sum_j |X_j W1[j,k]| + |H_k|)."""
    S1 = np.abs(X) @ np.abs(W1)
    return (S1 + np.abs(H)) @ np.abs(W2)


def hyperneat(gen, tr, n_grid: int, n_out: int, X: np.ndarray, dY: np.ndarray,
              thr: float = THRESHOLD) -> Dict[str, object]:
    """Whole pipeline for one CPPN: weights, substrate outputs, gradients."""
    grid = grid_coords(n_grid)
    outs = row_coords(n_out)
    raw1 = cppn_weights(gen, tr, grid, grid)
    raw2 = cppn_weights(gen, tr, grid, outs)
    W1, W2 = threshold(raw1, thr), threshold(raw2, thr)
    H, Y = substrate_forward(X, W1, W2)
    dW1, dW2 = substrate_backward(X, W2, H, dY)
    g1 = cppn_gradient(gen, tr, grid, grid, raw1, dW1, thr)
    g2 = cppn_gradient(gen, tr, grid, outs, raw2, dW2, thr)
    dw = {r: g1[0][r] + g2[0][r] for r in g1[0]}
    db = {r: g1[1][r] + g2[1][r] for r in g1[1]}
    return {"raw1": raw1, "raw2": raw2, "W1": W1, "W2": W2, "H": H, "Y": Y,
            "dW1": dW1, "dW2": dW2, "dw_cppn": dw, "db_cppn": db}


def substrate_genome_arrays(W1: np.ndarray, W2: np.ndarray) -> Tuple[list, list]:
    """The substrate as an ordinary genome (node rows, connection rows) with
    inputs 0..S1-1, outputs S1..S1+m-1, hidden nodes after them: every nonzero
    weight is an enabled connection; hidden nodes use tanh, outputs identity,
    all biases 0 and responses 1. Used to pin the substrate forward to the
    genome forward."""
    S1, S2 = W1.shape
    m = W2.shape[1]
    hid0 = S1 + m
    nodes = [[k, 0.0, 1.0, 0, 0] for k in range(S1)]
    nodes += [[S1 + j, 0.0, 1.0, 0, 0] for j in range(m)]          # identity
    nodes += [[hid0 + h, 0.0, 1.0, 2, 0] for h in range(S2)]       # tanh
    conns = []
    for i in range(S1):
        for h in range(S2):
            if W1[i, h] != 0.0:
                conns.append([i, hid0 + h, float(W1[i, h]), 1])
    for h in range(S2):
        for j in range(m):
            if W2[h, j] != 0.0:
                conns.append([hid0 + h, S1 + j, float(W2[h, j]), 1])
    return nodes, conns
