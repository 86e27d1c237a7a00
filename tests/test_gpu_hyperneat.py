"""GPU parity of the HyperNEAT path (tn_cppn_query, tn_substrate_forward)
against the float64 oracle.

CPPN values (before the threshold): the forward tolerance of test_gpu_forward,
|w - w_ref| <= 1e-5 * cond + 2^-100. Stored weights: bit-exact round to
nearest even of the GPU's own thresholded float32 value; threshold decisions
equal the oracle's except where |w_ref| lies within the forward tolerance of
the threshold (counted, not compared: both sides take the decision in their own
precision there).
Substrate: with the GPU's bfloat16 weights and inputs as exact float64 values
(their products are exact in float32), float32 accumulation of K = 1024 terms
errs by at most K * 2^-24 = 2^-14 times the sum of the terms' magnitudes, so
|h - tanh(z_ref)| <= 2^-14 * sum_s |x_s w_s| + 2^-21 (the last term: tanh's
own error from the hardware exp and reciprocal), and y against bf16(h) W2
within 2^-14 * sum_t |bf16(h_t) w_t|. End to end against the float64 oracle
with float64 weights (the GPU's threshold decisions): |y - y_ref| <= 2^-7 *
error_scale: the four bfloat16 roundings take at most 2^-8 of it (pinned in
test_oracle_hyperneat), the accumulations and the CPPN's float32 error (below
1e-5 relative) stay inside the remaining factor of two.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import host, to_device
from oracle import hyperneat as hn

pytestmark = pytest.mark.gpu
GRID, NOUT, THR = 32, 8, 0.2


def _bf16_bits(x):
    u = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    nan = np.isnan(np.asarray(x, np.float32))
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)
    r[nan] = 0x7FC0
    return r


def _bits16(t):
    return host(t.view(torch.int16)).view(np.uint16)


def _bf16_value(bits):
    return (bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def _query(P, seed=5):
    import paper_2504_08339_amd as tn
    pop = synth.cppn_population(seed=seed, P=P)
    dp = to_device(pop)
    tr = tn.transform(dp)
    w1t, w2t, r1, r2 = tn.cppn_query(dp, tr, GRID, NOUT, THR, raw=True)
    return tn, pop, dp, tr, w1t, w2t, r1, r2


def _check_genome(pop, g, r1, r2, w1b, w2b):
    gen = oracle.decode(pop, g)
    tr = oracle.transform(gen)
    grid, outs = hn.grid_coords(GRID), hn.row_coords(NOUT)
    ambiguous = 0
    for src_xy, dst_xy, raw, wb in ((grid, grid, r1[g], w1b[g]), (grid, outs, r2[g], w2b[g])):
        ref, cond = oracle.forward(gen, tr, hn.query_inputs(src_xy, dst_xy), with_cond=True)
        ref = ref[:, 0].reshape(len(src_xy), len(dst_xy)).T      # [t][s]
        cond = cond[:, 0].reshape(len(src_xy), len(dst_xy)).T
        tol = 1e-5 * cond + 2.0 ** -100
        if tr.status:
            assert np.isnan(raw).all()
            continue
        err = np.abs(raw.astype(np.float64) - ref)
        assert np.all(err <= tol), (g, float(err.max()))
        kept = np.where(np.abs(raw) < THR, np.float32(0), raw)
        assert np.array_equal(wb, _bf16_bits(kept))
        near = np.abs(np.abs(ref) - THR) <= tol
        ambiguous += int(near.sum())
        same = (np.abs(raw) < THR) == (np.abs(ref) < THR)
        assert np.all(same | near)
    return ambiguous


def test_cppn_query_matches_oracle():
    tn, pop, dp, tr, w1t, w2t, r1, r2 = _query(6)
    r1, r2 = host(r1), host(r2)
    w1b, w2b = _bits16(w1t), _bits16(w2t)
    assert w1b.shape == (6, 1024, 1024) and w2b.shape == (6, 8, 1024)
    amb = sum(_check_genome(pop, g, r1, r2, w1b, w2b) for g in range(pop.P))
    print("threshold decisions within tolerance of 0.2:", amb)
    assert (w1b != 0).any() and (w1b == 0).any()      # the threshold did something


def test_cppn_query_flagged_and_shape_errors():
    import paper_2504_08339_amd as tn
    from helpers import population_from_rows
    good = [[k, 0.0, 1.0, 0, 0] for k in range(5)] + [[5, 0.1, 1.0, 2, 0]]
    cyc = good + [[7, 0.0, 1.0, 2, 0], [8, 0.0, 1.0, 2, 0]]
    pop = population_from_rows([(good, [[0, 5, 1.0, 1], [4, 5, 0.5, 1]]),
                                (cyc, [[7, 8, 1.0, 1], [8, 7, 1.0, 1], [8, 5, 1.0, 1]])], 5, 1,
                               N_max=12, C_max=6)
    dp = to_device(pop)
    tr = tn.transform(dp)
    w1t, w2t, r1, r2 = tn.cppn_query(dp, tr, 8, 2, THR, raw=True)
    assert host(tr.status)[1] != 0
    assert np.isnan(host(r1)[1]).all() and np.all(_bits16(w1t)[1] == 0x7FC0)
    assert np.isfinite(host(r1)[0]).all()
    with pytest.raises(tn.TNError):
        tn.cppn_query(dp, tr, 6, 2, THR)               # 36 nodes: not a multiple of 64
    xor = to_device(synth.xor_population(P=2))
    with pytest.raises(tn.TNError):
        tn.cppn_query(xor, tn.transform(xor), 8, 2, THR)   # not a 5 -> 1 CPPN
    u1 = torch.zeros((2, 64, 64), device="cuda")
    u2 = torch.zeros((2, 2, 64), device="cuda")
    dW, db = tn.cppn_backward(dp, tr, u1, u2, 8, 2, THR)
    assert np.isnan(host(dW)[1]).all() and np.isnan(host(db)[1]).all()
    assert np.all(host(dW)[0] == 0.0) and np.all(host(db)[0] == 0.0)


def _substrate_case(P, B, shared):
    tn, pop, dp, tr, w1t, w2t = _query(P, seed=15)[:6]
    rng = np.random.default_rng(8)
    X = rng.standard_normal((B, GRID * GRID) if shared else (P, B, GRID * GRID)).astype(np.float32)
    xb = torch.from_numpy(X).cuda().to(torch.bfloat16)
    h, y = tn.substrate_forward(w1t, w2t, xb, GRID, NOUT, THR)
    return tn, pop, w1t, w2t, xb, host(h), host(y)


@pytest.mark.parametrize("shared", [True, False])
def test_substrate_forward_matches_oracle_on_gpu_weights(shared):
    tn, pop, w1t, w2t, xb, h, y = _substrate_case(4, 100, shared)
    W1 = _bf16_value(_bits16(w1t))          # [P][t][s]
    W2 = _bf16_value(_bits16(w2t))          # [P][j][t]
    Xv = _bf16_value(_bits16(xb))
    for g in range(pop.P):
        Xg = Xv if shared else Xv[g]
        Z = Xg @ W1[g].T
        S1 = np.abs(Xg) @ np.abs(W1[g]).T
        assert np.all(np.abs(h[g] - np.tanh(Z)) <= 2.0 ** -14 * S1 + 2.0 ** -21), g
        Hb = _bf16_value(_bf16_bits(h[g]))
        ref = Hb @ W2[g].T
        bound = 2.0 ** -14 * (np.abs(Hb) @ np.abs(W2[g]).T) + 1e-30
        assert np.all(np.abs(y[g] - ref) <= bound), g


def test_substrate_end_to_end_against_float64():
    """GPU outputs against the float64 pipeline (float64 CPPN weights with the
    GPU's threshold decisions, float64 inputs, no rounding)."""
    tn, pop, dp, tr, w1t, w2t, r1, r2 = _query(3, seed=25)
    rng = np.random.default_rng(9)
    X = rng.standard_normal((64, GRID * GRID)).astype(np.float32)
    xb = torch.from_numpy(X).cuda().to(torch.bfloat16)
    h, y = tn.substrate_forward(w1t, w2t, xb, GRID, NOUT, THR)
    y = host(y)
    r1, r2 = host(r1), host(r2)
    grid, outs = hn.grid_coords(GRID), hn.row_coords(NOUT)
    for g in range(pop.P):
        gen = oracle.decode(pop, g)
        otr = oracle.transform(gen)
        raw1 = hn.cppn_weights(gen, otr, grid, grid)      # [s][t]
        raw2 = hn.cppn_weights(gen, otr, grid, outs)
        W1 = np.where(np.abs(r1[g].T) < THR, 0.0, raw1)   # the GPU's decisions
        W2 = np.where(np.abs(r2[g].T) < THR, 0.0, raw2)
        H, Y = hn.substrate_forward(X.astype(np.float64), W1, W2)
        scale = hn.error_scale(X.astype(np.float64), W1, W2, H)
        assert np.all(np.abs(y[g] - Y) <= 2.0 ** -7 * scale), g


def test_full_size_sampled():
    """1000 CPPNs on the 32 x 32 / 32 x 32 / 8 substrate with 128 inputs per
    genome, as the benchmark runs it; two sampled genomes against the oracle."""
    import paper_2504_08339_amd as tn
    pop = synth.cppn_population()
    dp = to_device(pop)
    tr = tn.transform(dp)
    w1t, w2t = tn.cppn_query(dp, tr, GRID, NOUT, THR)
    X = torch.randn((pop.P, 128, GRID * GRID), generator=torch.Generator().manual_seed(5))
    xb = X.cuda().to(torch.bfloat16)
    h, y = tn.substrate_forward(w1t, w2t, xb, GRID, NOUT, THR)
    torch.cuda.synchronize()
    yh = host(y)
    assert np.isfinite(yh).all()
    W1 = w1t.float()
    W2 = w2t.float()
    Xv = xb.float()
    for g in (17, 803):
        ref = torch.tanh(Xv[g].double() @ W1[g].double().T)
        assert torch.all((h[g].double() - ref).abs() <= 2.0 ** -14 * (Xv[g].double().abs() @ W1[g].double().abs().T) + 2.0 ** -21)
        Hb = h[g].to(torch.bfloat16).double()
        refy = Hb @ W2[g].double().T
        assert torch.all((y[g].double() - refy).abs() <= 2.0 ** -14 * (Hb.abs() @ W2[g].double().abs().T) + 1e-30)
        # the sampled weights against the oracle's CPPN
        gen = oracle.decode(pop, g)
        otr = oracle.transform(gen)
        src = hn.grid_coords(GRID)[::97]
        ref_w = hn.cppn_weights(gen, otr, src, hn.grid_coords(GRID))    # [s][t]
        got = W1[g][:, ::97].cpu().numpy().T                          # [s][t]
        ok = (np.abs(np.abs(ref_w) - THR) > 1e-4)
        expect = _bf16_value(_bf16_bits(hn.threshold(ref_w).astype(np.float32)))
        assert np.all((np.abs(got - expect) <= 2.0 ** -7 * np.abs(expect)) | ~ok)   # one bf16 step


@pytest.mark.parametrize("shared", [True, False])
def test_substrate_backward_matches_oracle(shared):
    """Gradients of sum(dY * Y) against the oracle's substrate adjoint computed
    from the GPU's own h, weights and inputs. dw2t: float32 sums of B <= 128
    terms, |err| <= 2^-17 * sum_b |h dy|; dw1t: dZ rounded to bfloat16 (2^-9)
    plus float32 accumulation, |err| <= 2^-8 * sum_b |dz_b x_b|."""
    import paper_2504_08339_amd as tn
    P, B = 3, 100
    _, pop, w1t, w2t, xb, h, y = _substrate_case(P, B, shared)
    dy = np.random.default_rng(12).standard_normal((P, B, NOUT)).astype(np.float32)
    dw1t, dw2t = tn.substrate_backward(w2t, xb, torch.from_numpy(h).cuda(),
                                       torch.from_numpy(dy).cuda(), GRID, NOUT, THR)
    dw1t, dw2t = host(dw1t), host(dw2t)
    W2 = _bf16_value(_bits16(w2t))          # [P][j][t]
    Xv = _bf16_value(_bits16(xb))
    for g in range(P):
        Xg = Xv if shared else Xv[g]
        H = h[g].astype(np.float64)
        dY = dy[g].astype(np.float64)
        dW1, dW2 = hn.substrate_backward(Xg, W2[g].T, H, dY)      # [s][t], [t][j]
        b2 = 2.0 ** -17 * (np.abs(H).T @ np.abs(dY)) + 1e-30
        assert np.all(np.abs(dw2t[g].T - dW2) <= b2), g
        dZ = (dY @ W2[g]) * (1.0 - H * H)
        b1 = 2.0 ** -8 * (np.abs(Xg).T @ np.abs(dZ)) + 1e-30            # [s][t]
        assert np.all(np.abs(dw1t[g].T - dW1) <= b1), g


def _cppn_grad_case(grid, n_out, P, seed):
    import paper_2504_08339_amd as tn
    pop = synth.cppn_population(seed=seed, P=P)
    dp = to_device(pop)
    tr = tn.transform(dp)
    w1t, w2t, r1, r2 = tn.cppn_query(dp, tr, grid, n_out, THR, raw=True)
    S = grid * grid
    rng = np.random.default_rng(seed)
    u1 = rng.standard_normal((P, S, S)).astype(np.float32)
    u2 = rng.standard_normal((P, n_out, S)).astype(np.float32)
    dW, db = tn.cppn_backward(dp, tr, torch.from_numpy(u1).cuda(), torch.from_numpy(u2).cuda(),
                              grid, n_out, THR)
    return pop, host(r1), host(r2), u1, u2, host(dW), host(db)


def _check_cppn_grads(pop, grid, n_out, r1, r2, u1, u2, dW, db, genomes):
    """Against the oracle's CPPN adjoint with the GPU's threshold decisions:
    |g - g_ref| <= 1e-4 |g_ref| + 1e-5 max|g_ref| per genome (float32 sums
    over up to 2^20 queries of terms that carry the forward's 1e-5 error)."""
    src, outs = hn.grid_coords(grid), hn.row_coords(n_out)
    for g in genomes:
        gen = oracle.decode(pop, g)
        tr = oracle.transform(gen)
        if tr.status:
            assert np.isnan(dW[g]).all() and np.isnan(db[g]).all()
            continue
        a = hn.cppn_gradient(gen, tr, src, src, r1[g].T, u1[g].T.astype(np.float64))
        b = hn.cppn_gradient(gen, tr, src, outs, r2[g].T, u2[g].T.astype(np.float64))
        ref_w = np.zeros(pop.C_max)
        ref_b = np.zeros(pop.N_max)
        for row, val in a[0].items():
            ref_w[row] += val + b[0][row]
        for row, val in a[1].items():
            ref_b[row] += val + b[1][row]
        ref = np.concatenate([ref_w, ref_b])
        got = np.concatenate([dW[g], db[g]]).astype(np.float64)
        tol = 1e-4 * np.abs(ref) + 1e-5 * np.abs(ref).max()
        assert np.all(np.abs(got - ref) <= tol), (g, float(np.max(np.abs(got - ref) - tol)))


def test_cppn_backward_small_grid():
    pop, r1, r2, u1, u2, dW, db = _cppn_grad_case(8, 2, 8, 31)
    _check_cppn_grads(pop, 8, 2, r1, r2, u1, u2, dW, db, range(pop.P))
    dead = (pop.conn_in < 0) | (pop.conn_en == 0)
    assert np.all(dW[dead] == 0.0)
    assert np.all(db[pop.node_key < pop.n_in] == 0.0)


def test_cppn_backward_full_substrate():
    pop, r1, r2, u1, u2, dW, db = _cppn_grad_case(GRID, NOUT, 2, 41)
    _check_cppn_grads(pop, GRID, NOUT, r1, r2, u1, u2, dW, db, range(pop.P))


def test_cppn_backward_both_slot_forms_and_edge_limit():
    """CPPNs of 34 to 70 enabled in-edges: the compact form (at most 48
    in-edges) and the full one (49 to 64) against the oracle, NaN above the
    64 in-edges the adjoint holds."""
    import paper_2504_08339_amd as tn
    rng = np.random.default_rng(61)
    muts = np.array([30, 46, 50, 54, 58, 62, 75, 40])
    pop = synth.grow_population(8, 5, 1, 32, 128, muts, rng,
                                hidden_acts=("sin", "gaussian", "tanh", "abs"),
                                output_acts=("tanh",))
    edges = [int((pop.conn_rows(g)["en"] > 0).sum()) for g in range(pop.P)]
    assert min(edges) <= 48 and any(48 < e <= 64 for e in edges) and max(edges) > 64
    grid, n_out = 8, 2
    dp = to_device(pop)
    tr = tn.transform(dp)
    _, _, r1, r2 = tn.cppn_query(dp, tr, grid, n_out, THR, raw=True)
    S = grid * grid
    u1 = rng.standard_normal((pop.P, S, S)).astype(np.float32)
    u2 = rng.standard_normal((pop.P, n_out, S)).astype(np.float32)
    dW, db = tn.cppn_backward(dp, tr, torch.from_numpy(u1).cuda(), torch.from_numpy(u2).cuda(),
                              grid, n_out, THR)
    dW, db = host(dW), host(db)
    over = [g for g in range(pop.P) if edges[g] > 64]
    for g in over:
        assert np.isnan(dW[g]).all() and np.isnan(db[g]).all()
    _check_cppn_grads(pop, grid, n_out, host(r1), host(r2), u1, u2, dW, db,
                      [g for g in range(pop.P) if edges[g] <= 64])


def test_cppn_backward_through_the_substrate():
    """The whole chain: CPPN query -> substrate forward -> substrate backward ->
    CPPN adjoint, against the oracle's pipeline gradient (with the GPU's
    threshold decisions and the GPU's substrate gradients as upstream)."""
    import paper_2504_08339_amd as tn
    pop = synth.cppn_population(seed=51, P=2)
    dp = to_device(pop)
    tr = tn.transform(dp)
    grid, n_out = 8, 4
    w1t, w2t, r1, r2 = tn.cppn_query(dp, tr, grid, n_out, THR, raw=True)
    rng = np.random.default_rng(6)
    xb = torch.from_numpy(rng.standard_normal((32, grid * grid)).astype(np.float32)).cuda().to(torch.bfloat16)
    h, y = tn.substrate_forward(w1t, w2t, xb, grid, n_out)
    dy = torch.from_numpy(rng.standard_normal((2, 32, n_out)).astype(np.float32)).cuda()
    dw1t, dw2t = tn.substrate_backward(w2t, xb, h, dy, grid, n_out)
    dW, db = tn.cppn_backward(dp, tr, dw1t, dw2t, grid, n_out)
    _check_cppn_grads(pop, grid, n_out, host(r1), host(r2), host(dw1t), host(dw2t), host(dW),
                      host(db), range(pop.P))
