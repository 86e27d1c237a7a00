"""Pins of the HyperNEAT oracle: substrate geometry, a CPPN with a closed-form
output, the threshold boundary, the substrate forward against element-wise
sums and against the genome forward of the same network, both gradients
against central finite differences, and the bfloat16 error scale."""
import copy

import numpy as np

import oracle
import synth
from helpers import population_from_rows
from oracle import hyperneat as hn


def test_grid_and_row_coordinates():
    g = hn.grid_coords(32)
    assert g.shape == (1024, 2)
    assert tuple(g[0]) == (-1.0, -1.0) and tuple(g[31]) == (1.0, -1.0)
    assert tuple(g[32 * 31]) == (-1.0, 1.0) and tuple(g[1023]) == (1.0, 1.0)
    assert np.allclose(g[32 * 5 + 7], (-1 + 14 / 31, -1 + 10 / 31), rtol=0, atol=1e-15)
    o = hn.row_coords(8)
    assert np.allclose(o[:, 0], np.linspace(-1, 1, 8)) and np.all(o[:, 1] == 0)


def test_query_inputs_are_source_major():
    src = np.array([[0.1, 0.2], [0.3, 0.4]])
    dst = np.array([[-1.0, 0.5], [0.0, 0.25], [1.0, -0.5]])
    q = hn.query_inputs(src, dst)
    assert q.shape == (6, 5)
    for s in range(2):
        for t in range(3):
            assert np.array_equal(q[s * 3 + t], [*src[s], *dst[t], 1.0])


def _linear_cppn(a, b):
    """5 inputs wired straight to one tanh output: w = tanh(b + sum a_i q_i)."""
    nodes = [[k, 0.0, 1.0, 0, 0] for k in range(5)] + [[5, b, 1.0, 2, 0]]
    conns = [[k, 5, a[k], 1] for k in range(5)]
    pop = population_from_rows([(nodes, conns)], 5, 1)
    gen = oracle.decode(pop, 0)
    return gen, oracle.transform(gen), pop


def test_linear_cppn_closed_form():
    a = [0.7, -1.3, 0.4, 2.1, -0.25]
    gen, tr, pop = _linear_cppn(a, 0.3)
    a32 = pop.conn_w[0, :5].astype(np.float64)
    b32 = float(pop.node_bias[0, 5])
    src, dst = hn.grid_coords(4), hn.row_coords(3)
    W = hn.cppn_weights(gen, tr, src, dst)
    for s in range(16):
        for t in range(3):
            z = b32 + a32[0] * src[s, 0] + a32[1] * src[s, 1] + a32[2] * dst[t, 0] \
                + a32[3] * dst[t, 1] + a32[4]
            assert abs(W[s, t] - np.tanh(z)) <= 1e-15


def test_threshold_boundary():
    w = np.array([0.2, -0.2, 0.19999999, -0.19999999, 0.5, 0.0, -3.0])
    assert np.array_equal(hn.threshold(w), [0.2, -0.2, 0.0, 0.0, 0.5, 0.0, -3.0])


def test_substrate_forward_elementwise():
    rng = np.random.default_rng(0)
    X, W1, W2 = rng.standard_normal((3, 5)), rng.standard_normal((5, 4)), rng.standard_normal((4, 2))
    H, Y = hn.substrate_forward(X, W1, W2)
    for b in range(3):
        for h in range(4):
            z = 0.0
            for i in range(5):
                z += X[b, i] * W1[i, h]
            assert abs(H[b, h] - np.tanh(z)) <= 1e-14
        for j in range(2):
            y = 0.0
            for h in range(4):
                y += np.tanh(sum(X[b, i] * W1[i, h] for i in range(5))) * W2[h, j]
            assert abs(Y[b, j] - y) <= 1e-13


def test_substrate_equals_genome_forward():
    """The substrate encoded by a generated CPPN, built as an ordinary genome
    (every surviving weight a connection), gives the same outputs through the
    genome forward."""
    pop = synth.cppn_population(P=6)
    rng = np.random.default_rng(3)
    grid, outs = hn.grid_coords(3), hn.row_coords(2)
    checked = 0
    for g in range(pop.P):
        gen = oracle.decode(pop, g)
        tr = oracle.transform(gen)
        W1 = hn.threshold(hn.cppn_weights(gen, tr, grid, grid)).astype(np.float32).astype(np.float64)
        W2 = hn.threshold(hn.cppn_weights(gen, tr, grid, outs)).astype(np.float32).astype(np.float64)
        nodes, conns = hn.substrate_genome_arrays(W1, W2)
        if not conns:
            continue
        sp = population_from_rows([(nodes, conns)], 9, 2)
        sg = oracle.decode(sp, 0)
        st = oracle.transform(sg)
        X = rng.standard_normal((7, 9))
        Yg = oracle.forward(sg, st, X)
        _, Ys = hn.substrate_forward(X, W1, W2)
        np.testing.assert_allclose(Yg, Ys, rtol=1e-12, atol=1e-12)
        checked += 1
    assert checked >= 4


def test_substrate_backward_finite_differences():
    rng = np.random.default_rng(1)
    X, W1, W2 = rng.standard_normal((4, 5)), rng.standard_normal((5, 3)), rng.standard_normal((3, 2))
    dY = rng.standard_normal((4, 2))
    H, _ = hn.substrate_forward(X, W1, W2)
    dW1, dW2 = hn.substrate_backward(X, W2, H, dY)

    def L(a, b):
        return float(np.sum(dY * hn.substrate_forward(X, a, b)[1]))
    h = 1e-6
    for M, dM, which in ((W1, dW1, 0), (W2, dW2, 1)):
        for idx in np.ndindex(M.shape):
            P, Q = M.copy(), M.copy()
            P[idx] += h
            Q[idx] -= h
            fd = (L(P, W2) - L(Q, W2)) / (2 * h) if which == 0 else (L(W1, P) - L(W1, Q)) / (2 * h)
            assert abs(dM[idx] - fd) <= 1e-7 * max(1.0, abs(fd)), (which, idx)


def test_cppn_gradient_finite_differences():
    """d(sum dY * Y)/d(CPPN weights and biases) through thresholded weights,
    against central differences; perturbations that move a weight across the
    threshold are excluded and counted."""
    pop = synth.cppn_population(P=3, seed=9)
    rng = np.random.default_rng(4)
    n_grid, n_out = 3, 2
    X = rng.standard_normal((5, n_grid * n_grid))
    dY = rng.standard_normal((5, n_out))
    grid, outs = hn.grid_coords(n_grid), hn.row_coords(n_out)
    h = 1e-6
    compared = crossed = 0
    for g in range(pop.P):
        gen = oracle.decode(pop, g)
        tr = oracle.transform(gen)
        res = hn.hyperneat(gen, tr, n_grid, n_out, X, dY)

        def loss_and_raw(gm):
            tm = oracle.transform(gm)
            r = hn.hyperneat(gm, tm, n_grid, n_out, X, dY)
            return float(np.sum(dY * r["Y"])), r["raw1"], r["raw2"]
        params = [("w", i) for i, c in enumerate(gen.conns) if c.enabled]
        params += [("b", k) for k in gen.nodes if k >= gen.n_in]
        for kind, key in params:
            gp, gm = copy.deepcopy(gen), copy.deepcopy(gen)
            if kind == "w":
                gp.conns[key].w += h
                gm.conns[key].w -= h
                got = res["dw_cppn"][gen.conns[key].row]
            else:
                gp.nodes[key].bias += h
                gm.nodes[key].bias -= h
                got = res["db_cppn"][gen.nodes[key].row]
            lp, r1p, r2p = loss_and_raw(gp)
            lm, r1m, r2m = loss_and_raw(gm)
            flips = any(np.any((np.abs(a) < hn.THRESHOLD) != (np.abs(b) < hn.THRESHOLD))
                        for a, b in ((r1p, r1m), (r2p, r2m)))
            if flips:
                crossed += 1
                continue
            fd = (lp - lm) / (2 * h)
            assert abs(got - fd) <= 1e-5 * max(1.0, abs(fd)), (g, kind, key, got, fd)
            compared += 1
    assert compared >= 20


def _bf16(x):
    """Round float32 to bfloat16, to nearest even (kept in float32 storage)."""
    u = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def test_bf16_rounding_stays_within_error_scale():
    """Rounding W1, W2, X and H to bfloat16 (relative error <= 2^-9 each) moves
    Y by at most 2^-7 * error_scale, the bound the GPU parity test uses."""
    rng = np.random.default_rng(7)
    X = rng.standard_normal((16, 64))
    W1 = hn.threshold(rng.uniform(-1, 1, (64, 64)))
    W2 = hn.threshold(rng.uniform(-1, 1, (64, 8)))
    H, Y = hn.substrate_forward(X, W1, W2)
    scale = hn.error_scale(X, W1, W2, H)
    Xb, W1b, W2b = (_bf16(a).astype(np.float64) for a in (X, W1, W2))
    Hb = _bf16(np.tanh(Xb @ W1b)).astype(np.float64)
    Yb = Hb @ W2b
    assert np.all(np.abs(Yb - Y) <= 2.0 ** -7 * scale)
    assert np.array_equal(_bf16(np.float32([1.0, 1.00390625, 1.01171875])),
                          np.float32([1.0, 1.0, 1.015625]))   # ties to even
