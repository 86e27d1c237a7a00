"""GPU parity of the batched plan (tn_plan_*): the persistent, graph-captured
form and the plain per-bucket form give the bits of tn_forward, on uneven
ragged populations, across graph replays, pointer changes, tile changes and
tuning; sampled genomes against the float64 oracle (tolerance as in
test_gpu_forward)."""
import os

import numpy as np
import pytest
import torch

import synth
from gpu_util import host, tensor, to_device
from test_gpu_forward import check

pytestmark = pytest.mark.gpu


def _bits(x):
    return host(x).view(np.uint32)


def _setup(P, B, seed=41):
    import paper_2504_08339_amd as tn
    pop = synth.batching_population(P=P)
    dp = to_device(pop)
    tr = tn.transform(dp)
    obs = synth.normal_obs(P, B, pop.n_in, seed)
    return tn, pop, dp, tr, obs


@pytest.mark.parametrize("B", [150, 300, 50])
def test_plan_buckets_cover_population_and_match_forward(B):
    """Register buckets hold two tiles per wavefront (150 observations), four
    (300, the last wavefront of a genome half empty) or one (50)."""
    tn, pop, dp, tr, obs = _setup(600, B)
    xt = tensor(obs)
    plan = tn.Plan(dp, tr, B)
    bks = plan.buckets()
    assert sum(b["count"] for b in bks) == pop.P
    engines = {b["engine"] for b in bks}
    assert engines == {tn.TN_ENGINE_REG, tn.TN_ENGINE_LDS}
    ref = tn.forward(dp, tr, xt)
    a = plan.forward(xt)
    b = plan.forward_buckets(xt)
    assert np.array_equal(_bits(a), _bits(ref))
    assert np.array_equal(_bits(b), _bits(ref))
    check(pop, obs, host(a), list(range(0, pop.P, 37)))


def test_graph_replays_and_pointer_changes():
    tn, pop, dp, tr, obs = _setup(300, 100)
    xt = tensor(obs)
    plan = tn.Plan(dp, tr, 100)
    ref = _bits(tn.forward(dp, tr, xt))
    out = torch.empty((pop.P, 100, pop.n_out), dtype=torch.float32, device="cuda")
    for _ in range(4):                         # replays with eager work in between
        out.fill_(float("nan"))
        plan.forward(xt, out)
        torch.cuda.synchronize()
        assert np.array_equal(_bits(out), ref)
        _ = (xt * 2.0).sum().item()
    out2 = torch.empty_like(out)               # new output buffer: captured again
    plan.forward(xt, out2)
    assert np.array_equal(_bits(out2), ref)
    xt2 = xt.clone()                           # new observation buffer
    plan.forward(xt2, out)
    assert np.array_equal(_bits(out), ref)


def test_shared_observations_and_tile_changes():
    tn, pop, dp, tr, _ = _setup(250, 70)
    X = synth.normal_obs(1, 70, pop.n_in, 5)[0]
    xt = tensor(X)
    plan = tn.Plan(dp, tr, 70)
    ref = _bits(tn.forward(dp, tr, xt))
    for i, b in enumerate(plan.buckets()):
        # sixteen wavefronts: LDS engine at one observation per lane only
        bad = (1, 16) if b["engine"] == tn.TN_ENGINE_REG else (2, 16)
        with pytest.raises(tn.TNError):
            plan.set_tile(i, *bad)
        for K, W in ((1, 1), (1, 8)) if b["engine"] == tn.TN_ENGINE_REG else ((2, 2), (4, 1), (1, 8),
                                                                            (1, 16)):
            try:
                plan.set_tile(i, K, W)
            except tn.TNError:
                continue                       # tile does not fit this bucket's rows
            assert np.array_equal(_bits(plan.forward(xt)), ref), (i, K, W)
            assert np.array_equal(_bits(plan.forward_buckets(xt)), ref), (i, K, W)


def test_tune_and_cache(tmp_path):
    tn, pop, dp, tr, obs = _setup(400, 64)
    xt = tensor(obs)
    cache = str(tmp_path / "tiles.txt")
    plan = tn.Plan(dp, tr, 64)
    ref = _bits(tn.forward(dp, tr, xt))
    plan.tune(xt, tune_cache=cache)
    assert os.path.exists(cache)
    assert np.array_equal(_bits(plan.forward(xt)), ref)
    tuned = plan.buckets()
    again = tn.Plan(dp, tr, 64, tune_cache=cache)
    assert [(b["obs_per_lane"], b["waves"]) for b in again.buckets()] == \
        [(b["obs_per_lane"], b["waves"]) for b in tuned]
    assert np.array_equal(_bits(again.forward(xt)), ref)


def test_flagged_and_empty():
    import paper_2504_08339_amd as tn
    from test_gpu_transform import _malformed
    pop = _malformed()
    dp = to_device(pop)
    tr = tn.transform(dp)
    X = tensor(np.random.default_rng(1).standard_normal((5, 2)).astype(np.float32))
    plan = tn.Plan(dp, tr, 5)
    y = host(plan.forward(X))
    st = host(tr.status)[:pop.P]
    assert np.isnan(y[st != 0]).all() and np.isfinite(y[st == 0]).all()
    assert np.array_equal(y.view(np.uint32), _bits(tn.forward(dp, tr, X)))
    empty = synth.subset(synth.batching_population(P=10), [])
    de = to_device(empty)
    te = tn.transform(de)
    pe = tn.Plan(de, te, 5)
    assert pe.buckets() == []
    assert pe.forward(tensor(np.zeros((5, 27), np.float32))).shape == (0, 5, 8)


def test_full_batching_workload_all_genomes():
    """10000 uneven genomes x 256 observations, the benchmark's configuration
    (a tuned plan): persistent graph form equals the per-bucket form bitwise;
    every output of every genome against the oracle, with the worst
    |err| / cond reported per plan bucket."""
    import oracle_pool
    import paper_2504_08339_amd as tn
    from gpu_util import bucket_members
    from test_gpu_forward import ABS_FLOOR, RTOL
    pop = synth.batching_population()
    obs = synth.normal_obs(pop.P, 256, pop.n_in, 103)
    dp = to_device(pop)
    tr = tn.transform(dp)
    xt = tensor(obs)
    plan = tn.Plan(dp, tr, 256)
    plan.tune(xt)
    a = plan.forward(xt)
    b = plan.forward_buckets(xt)
    assert np.array_equal(_bits(a), _bits(b))
    Y = host(a).astype(np.float64)
    ref, cond, st = oracle_pool.forward_reference("batching", pop.P)
    assert np.isnan(Y[st != 0]).all()
    members = bucket_members(pop, tr, plan.buckets())
    assert sorted(np.concatenate(members).tolist()) == list(range(pop.P))
    for i, (bk, m) in enumerate(zip(plan.buckets(), members)):
        m = m[st[m] == 0]
        err = np.abs(Y[m] - ref[m])
        bad = err > RTOL * cond[m] + ABS_FLOOR
        assert not bad.any(), (i, int(bad.sum()))
        pos = cond[m] > 0
        worst = float((err[pos] / cond[m][pos]).max()) if pos.any() else 0.0
        print(f"bucket {i} engine {bk['engine']} rows<={bk['rows_class']} "
              f"{len(m)} genomes: worst |err|/cond {worst:.3e}")


def test_buckets_one_by_one_rebuild_the_outputs():
    tn, pop, dp, tr, obs = _setup(350, 90)
    xt = tensor(obs)
    plan = tn.Plan(dp, tr, 90)
    ref = _bits(tn.forward(dp, tr, xt))
    for persistent in (True, False):
        out = torch.full((pop.P, 90, pop.n_out), float("nan"), device="cuda")
        for i in range(len(plan.buckets())):
            plan.forward_bucket(i, xt, out, persistent)
        assert np.array_equal(_bits(out), ref), persistent
