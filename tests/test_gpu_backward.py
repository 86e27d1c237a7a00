"""GPU parity of the adjoint (tn_backward, tn_forward_backward_mse) against the
float64 oracle gradient and float64 central finite differences.

Tolerances (per genome): against the oracle gradient
    |g - g_ref| <= 1e-5 * |g_ref| + 1e-6 * max|g_ref|
and against finite differences (h = 1e-6)
    |g - fd| <= 1e-4 * |fd| + 1e-6 * max|fd|.
The absolute term is the float32 error of a batch sum whose terms cancel: its
size is a few unit roundoffs times sqrt(B) times a typical term, far below
1e-6 of the genome's largest gradient component, which sums B terms of one sign.
"""
import copy

import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import host, tensor, to_device

pytestmark = pytest.mark.gpu


def _cfg3(P):
    pop = synth.differentiation_population(P=P)
    X = synth.uniform_inputs(1024, 4, synth.CONFIG_SEEDS["differentiation"] + 100)
    T = synth.target_mlp(X, 32, 2, synth.CONFIG_SEEDS["differentiation"] + 200)
    return pop, X, T


def _close(g, ref, rel, absfrac):
    scale = np.max(np.abs(ref)) if ref.size else 0.0
    bad = np.abs(g - ref) > rel * np.abs(ref) + absfrac * scale
    return not bad.any(), (np.abs(g - ref) - rel * np.abs(ref)).max() if ref.size else 0.0


def check_grads(pop, dW, db, ref_dW, ref_db, genomes):
    for a, g in enumerate(genomes):
        st = oracle.transform(oracle.decode(pop, g)).status
        if st:
            assert np.isnan(dW[g]).all() and np.isnan(db[g]).all()
            continue
        ref = np.concatenate([ref_dW[a], ref_db[a]])
        got = np.concatenate([dW[g], db[g]]).astype(np.float64)
        ok, worst = _close(got, ref, 1e-5, 1e-6)
        assert ok, (g, worst)


def gpu_mse(pop, X, T):
    import paper_2504_08339_amd as tn
    dp = to_device(pop)
    tr = tn.transform(dp)
    loss, dW, db = tn.forward_backward_mse(dp, tr, tensor(X), tensor(T))
    return host(loss), host(dW), host(db)


def oracle_mse_grads(pop, X, T, genomes):
    dWs, dbs, losses = [], [], []
    for g in genomes:
        gen = oracle.decode(pop, g)
        tr = oracle.transform(gen)
        Xg = X if X.ndim == 2 else X[g]
        Tg = T if T.ndim == 2 else T[g]
        Y = oracle.forward(gen, tr, Xg)
        dY = 2.0 * (Y - Tg) / Y.size
        w, b = oracle.backward(gen, tr, Xg, dY)
        dW = np.zeros(pop.C_max)
        db = np.zeros(pop.N_max)
        for r, val in w.items():
            dW[r] = val
        for r, val in b.items():
            db[r] = val
        dWs.append(dW)
        dbs.append(db)
        losses.append(float(np.mean((Y - Tg) ** 2)))
    return np.array(losses), np.array(dWs), np.array(dbs)


def test_register_adjoint_limits_and_lds_fallback():
    """Genomes of 15 to 85 enabled in-edges, on both sides of the
    register-file adjoint's limits (at most 48 positions and 64 in-edges;
    larger ones go to the LDS kernel), against the oracle."""
    rng = np.random.default_rng(17)
    muts = np.array([10, 20, 30, 40, 45, 50, 55, 60, 70, 90, 25, 35])
    pop = synth.grow_population(len(muts), 4, 2, 64, 256, muts, rng, hidden_acts=("tanh",),
                                output_acts=("identity",), disable_p=0.1)
    sizes = []
    for g in range(pop.P):
        n = int((pop.node_rows(g)["key"] >= 0).sum())
        e = int((pop.conn_rows(g)["en"] > 0).sum())
        sizes.append((n, e))
    fits = [n <= 48 and e <= 64 for n, e in sizes]
    assert any(fits) and not all(fits) and any(48 < e <= 64 for _, e in sizes), sizes
    X = synth.uniform_inputs(300, 4, 23)
    T = synth.target_mlp(X, 16, 2, 24)
    loss, dW, db = gpu_mse(pop, X, T)
    ref_loss, ref_dW, ref_db = oracle_mse_grads(pop, X, T, range(pop.P))
    check_grads(pop, dW, db, ref_dW, ref_db, range(pop.P))


def test_lds_adjoint_beyond_device_lds():
    """N_max = 400: the LDS adjoint's N_max rows of values and gradients exceed
    the device's LDS. The call still succeeds; genomes within the register-file
    adjoint's limits get their gradients, the others NaN."""
    rng = np.random.default_rng(29)
    muts = np.array([10, 15, 20, 25, 90, 30, 95, 12])
    small = synth.grow_population(len(muts), 4, 2, 64, 256, muts, rng, hidden_acts=("tanh",),
                                  output_acts=("identity",), disable_p=0.1)
    pop = synth.to_padded(synth.to_ragged(small), N_max=400, C_max=256)
    fits = []
    for g in range(pop.P):
        n = int((pop.node_rows(g)["key"] >= 0).sum())
        e = int((pop.conn_rows(g)["en"] > 0).sum())
        fits.append(n <= 48 and e <= 64)
    assert any(fits) and not all(fits)
    X = synth.uniform_inputs(200, 4, 31)
    T = synth.target_mlp(X, 16, 2, 32)
    loss, dW, db = gpu_mse(pop, X, T)
    ok = [g for g in range(pop.P) if fits[g]]
    _, rW, rb = oracle_mse_grads(pop, X, T, ok)
    check_grads(pop, dW, db, rW, rb, ok)
    for g in range(pop.P):
        if not fits[g]:
            assert np.isnan(dW[g]).all() and np.isnan(db[g]).all() and np.isnan(loss[g])


def test_mse_gradients_match_oracle():
    pop, X, T = _cfg3(96)
    loss, dW, db = gpu_mse(pop, X, T)
    g = list(range(pop.P))
    rl, rW, rb = oracle_mse_grads(pop, X, T, g)
    np.testing.assert_allclose(loss, rl, rtol=1e-5, atol=0)
    check_grads(pop, dW, db, rW, rb, g)


def test_full_size_all_genomes():
    """4096 genomes x 1024 samples in the benchmark's launch configuration; the
    loss and every gradient of every genome against the oracle gradient
    (computed in parallel worker processes); the worst error, relative to the
    bar's scale, is reported."""
    import oracle_pool
    pop, X, T = _cfg3(4096)
    loss, dW, db = gpu_mse(pop, X, T)
    assert np.isfinite(loss).all()
    rl, rW, rb, st = oracle_pool.mse_grad_reference("differentiation", pop.P)
    assert not st.any()
    np.testing.assert_allclose(loss, rl, rtol=1e-5, atol=0)
    got = np.concatenate([dW, db], axis=1).astype(np.float64)
    ref = np.concatenate([rW, rb], axis=1)
    scale = np.abs(ref).max(axis=1, keepdims=True)
    err = np.abs(got - ref)
    bound = 1e-5 * np.abs(ref) + 1e-6 * scale
    assert not (err > bound).any(), int((err > bound).sum())
    # achieved: the error in units of the genome's largest gradient component
    # and, where the reference is not tiny, relative to the component itself
    big = np.abs(ref) > 1e-3 * scale
    print(f"differentiation 4096 genomes: worst |err|/max|g| {float((err / scale).max()):.3e}, "
          f"worst relative error on components above 1e-3 max|g| "
          f"{float((err[big] / np.abs(ref[big])).max()):.3e}")


def _loss64(gen, X, T):
    Y = oracle.forward(gen, oracle.transform(gen), X)
    return float(np.mean((Y - T) ** 2))


def test_finite_differences_64_genomes():
    """Every enabled weight and every non-input bias of 64 genomes against float64
    central differences of the oracle's loss, h = 1e-6."""
    pop, X, T = _cfg3(64)
    X64, T64 = X.astype(np.float64), T.astype(np.float64)
    _, dW, db = gpu_mse(pop, X, T)
    h = 1e-6
    n_params = 0
    for g in range(pop.P):
        gen = oracle.decode(pop, g)
        fds, got = [], []
        for i, c in enumerate(gen.conns):
            if not c.enabled:
                continue
            gp, gm = copy.deepcopy(gen), copy.deepcopy(gen)
            gp.conns[i].w += h
            gm.conns[i].w -= h
            fds.append((_loss64(gp, X64, T64) - _loss64(gm, X64, T64)) / (2 * h))
            got.append(dW[g, c.row])
        for k, node in gen.nodes.items():
            if k < pop.n_in:
                continue
            gp, gm = copy.deepcopy(gen), copy.deepcopy(gen)
            gp.nodes[k].bias += h
            gm.nodes[k].bias -= h
            fds.append((_loss64(gp, X64, T64) - _loss64(gm, X64, T64)) / (2 * h))
            got.append(db[g, node.row])
        fds, got = np.array(fds), np.array(got, np.float64)
        ok, worst = _close(got, fds, 1e-4, 1e-6)
        assert ok, (g, worst)
        n_params += len(fds)
    assert n_params > 1500


def test_given_upstream_gradient_all_functions():
    """tn_backward with a seeded dY, every activation and aggregation, random
    responses, batch not a multiple of 64."""
    import paper_2504_08339_amd as tn
    rng = np.random.default_rng(11)
    pop = synth.cppn_population(P=60, seed=91)
    valid = pop.node_key >= 0
    pop.node_act[valid] = rng.integers(0, 7, size=int(valid.sum()))
    pop.node_agg[valid] = rng.integers(0, 6, size=int(valid.sum()))
    pop.node_resp[valid] = rng.uniform(-2, 2, size=int(valid.sum())).astype(np.float32)
    B = 150
    X = rng.uniform(-1.5, 1.5, size=(pop.P, B, pop.n_in)).astype(np.float32)
    dY = rng.standard_normal((pop.P, B, pop.n_out)).astype(np.float32)
    dp = to_device(pop)
    tr = tn.transform(dp)
    dW, db = tn.backward(dp, tr, tensor(X), tensor(dY))
    dW, db = host(dW), host(db)
    rW, rb = oracle.backward_population(pop, X, dY)
    check_grads(pop, dW, db, rW, rb, list(range(pop.P)))


def test_zero_rows_flagged_and_deterministic():
    import paper_2504_08339_amd as tn
    from test_gpu_transform import _malformed
    pop, X, T = _cfg3(40)
    _, dW, db = gpu_mse(pop, X, T)
    dead = (pop.conn_in < 0) | (pop.conn_en == 0)
    assert np.all(dW[dead] == 0.0)
    assert np.all(db[(pop.node_key < pop.n_in)] == 0.0)
    _, dW2, db2 = gpu_mse(pop, X, T)
    assert np.array_equal(dW.view(np.uint32), dW2.view(np.uint32))
    assert np.array_equal(db.view(np.uint32), db2.view(np.uint32))
    bad = _malformed()
    Xb = np.random.default_rng(2).standard_normal((70, 2)).astype(np.float32)
    Tb = np.zeros((70, 1), np.float32)
    dpb = to_device(bad)
    trb = tn.transform(dpb)
    loss, dWb, dbb = tn.forward_backward_mse(dpb, trb, tensor(Xb), tensor(Tb))
    st = host(trb.status)
    loss, dWb, dbb = host(loss), host(dWb), host(dbb)
    for g in range(bad.P):
        if st[g]:
            assert np.isnan(loss[g]) and np.isnan(dWb[g]).all() and np.isnan(dbb[g]).all()
        else:
            assert np.isfinite(loss[g])


def test_ragged_equals_padded():
    pop, X, T = _cfg3(50)
    rag = synth.to_ragged(pop)
    l1, w1, b1 = gpu_mse(pop, X, T)
    l2, w2, b2 = gpu_mse(rag, X, T)
    assert np.array_equal(l1.view(np.uint32), l2.view(np.uint32))
    for g in range(pop.P):
        cv = np.flatnonzero(pop.conn_in[g] >= 0)
        nv = np.flatnonzero(pop.node_key[g] >= 0)
        cs = slice(int(rag.conn_off[g]), int(rag.conn_off[g + 1]))
        ns = slice(int(rag.node_off[g]), int(rag.node_off[g + 1]))
        assert np.array_equal(w1[g][cv], w2[cs])
        assert np.array_equal(b1[g][nv], b2[ns])


def test_autograd_function():
    import paper_2504_08339_amd as tn
    pop, X, T = _cfg3(16)
    dp = to_device(pop)
    w = dp.t["conn_w"].clone().requires_grad_(True)
    b = dp.t["node_bias"].clone().requires_grad_(True)
    Xt, Tt = tensor(X), tensor(T)
    y = tn.TNForward.apply(dp, Xt, w, b)
    loss = ((y - Tt.unsqueeze(0)) ** 2).mean(dim=(1, 2)).sum()
    loss.backward()
    tr = tn.transform(dp)
    _, dW, db = tn.forward_backward_mse(dp, tr, Xt, Tt)
    np.testing.assert_allclose(host(w.grad), host(dW), rtol=1e-5, atol=1e-7)
    np.testing.assert_allclose(host(b.grad), host(db), rtol=1e-5, atol=1e-7)
