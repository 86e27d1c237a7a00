#!/usr/bin/env python3
"""Throughput of the population-evaluation hot path on one MI355X.

Prints ONE JSON line. A step is one pass of the hot path over one batch of
synthetic input, with every input already resident in device memory.

Headline workload (`value`): uneven-size batching, 10,000 genomes with
log-uniform 10..500 hidden nodes and 2..4x as many connections (at most 2000),
27 inputs -> 8 outputs, ragged layout, 256 N(0,1) observations per genome:
one step = the batched forward of the whole population by a tuned plan, its
length buckets run as persistent kernels captured in one hipGraph
(2.56e6 genome-forward passes). The same plan's plain form (one ordinary
launch per bucket) is timed over the same number of steps for the comparison.

Beside it (`workloads`), each with its own timed steps and roofline:
  control          1000 genomes 17 -> 6 (N_max 64, C_max 256), 1000 obs each:
                   transform + forward + 1000 x 1000 compatibility distance;
  differentiation  4096 genomes 4 -> 2, 1024 shared samples: forward + adjoint
                   with the fused MSE loss;
  hyperneat        1000 CPPNs on a 32x32 / 32x32 / 8 grid substrate, 128 obs per
                   genome: CPPN query + substrate forward + substrate backward +
                   CPPN adjoint.

`value` is genome-forward passes per second (P * B per step / time per step).
The roofline object is for the dominant kernel of the headline step: every
bucket's persistent kernel is also launched alone, bracketed by HIP events on
the stream it runs on, and the slowest one's algorithmic bytes (observations
read, outputs written and the program words its genomes read, counted from
the actual population) over its average duration give `achieved`. The CPU
oracle is timed on a bounded sample for `cpu_baseline`.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("genome-forward-passes/s (pop×obs) + % HBM roofline; "
          "batched-persistent vs plain launch")
HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0


def _args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="rough budget of the CPU-oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only-headline", action="store_true",
                    help="skip the other workloads")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one 1 GiB device copy (counter calibration under rocprofv3)")
    return ap.parse_args()


def _log(msg):
    print(f"bench: {msg}", file=sys.stderr, flush=True)


class Timer:
    """HIP events around calls on torch's current stream (the stream every
    library call is launched on)."""

    def __init__(self, torch):
        self.torch = torch
        self.pairs = {}

    def __call__(self, name, fn, *a, **k):
        ev0 = self.torch.cuda.Event(enable_timing=True)
        ev1 = self.torch.cuda.Event(enable_timing=True)
        ev0.record()
        r = fn(*a, **k)
        ev1.record()
        self.pairs.setdefault(name, []).append((ev0, ev1))
        return r

    def mean_ms(self):
        return {n: sum(a.elapsed_time(b) for a, b in v) / len(v) for n, v in self.pairs.items()}


def timed_steps(torch, step, steps, warmup):
    """Warm-up steps, then exactly `steps` timed steps between synchronisations;
    returns (ms per step by the host clock, per-call mean ms by HIP events)."""
    t = Timer(torch)
    for _ in range(warmup):
        step(t)
    torch.cuda.synchronize()
    t = Timer(torch)
    t0 = time.perf_counter()
    for _ in range(steps):
        step(t)
    torch.cuda.synchronize()
    return 1e3 * (time.perf_counter() - t0) / steps, t.mean_ms()


def device_population(torch, tn, pop):
    arrays = {k: getattr(pop, k) for k in ("node_key", "node_bias", "node_resp", "node_act",
                                           "node_agg", "conn_in", "conn_out", "conn_w", "conn_en")}
    kw = {}
    if pop.ragged:
        kw = {"node_off": pop.node_off, "conn_off": pop.conn_off}
    return tn.Population.from_numpy(pop.n_in, pop.n_out, pop.N_max, pop.C_max, arrays,
                                    device="cuda", **kw)


def genome_sizes(torch, pop, tr):
    """(n_valid, enabled edges) per genome, read back from the transformation."""
    import numpy as np
    torch.cuda.synchronize()
    nv = tr.n_valid.cpu().numpy()[:pop.P].astype(np.int64)
    rp = tr.row_ptr.cpu().numpy()
    if pop.ragged:
        base = pop.node_off[:pop.P] + np.arange(pop.P)
    else:
        base = np.arange(pop.P) * (pop.N_max + 1)
    return nv, rp[base + nv].astype(np.int64)


# ------------------------------------------------------------------ batching

def batching(torch, tn, synth, args):
    import numpy as np
    pop = synth.batching_population()
    B = 256
    obs_np = synth.normal_obs(pop.P, B, pop.n_in, synth.CONFIG_SEEDS["batching"] + 100)
    dp = device_population(torch, tn, pop)
    obs = torch.from_numpy(obs_np).cuda()
    tr = tn.transform(dp)
    out = torch.empty((pop.P, B, pop.n_out), dtype=torch.float32, device="cuda")
    _log("batching: plan + tuning")
    plan = tn.Plan(dp, tr, B)
    plan.tune(obs, out)
    buckets = plan.buckets()
    nv, ne = genome_sizes(torch, pop, tr)
    I, O = pop.n_in, pop.n_out

    # algorithmic bytes per genome: observations in, outputs out, and the
    # program words the engine reads (register engine: 16 B per position and
    # 8 B per edge; LDS engine: row_ptr, level, fn, bias, resp, row 24 B per
    # position + 8 B per edge), plus the io positions
    prog_rows = tr.prog_rows.cpu().numpy()[:pop.P]
    reg = prog_rows <= 200
    per_genome = (4 * B * (I + O) + np.where(reg, 16 * nv, 24 * nv + 4) + 8 * ne
                  + 4 * (I + O) + 12)
    total_bytes = int(per_genome.sum())
    lists = bucket_members(pop, tr, buckets)
    bucket_bytes = [int(per_genome[m].sum()) for m in lists]

    _log("batching: persistent graph steps")
    graph_ms, _ = timed_steps(torch, lambda t: t("graph", plan.forward, obs, out),
                              args.steps, args.warmup)
    _log("batching: plain per-bucket steps")
    plain_ms, _ = timed_steps(torch, lambda t: t("plain", plan.forward_buckets, obs, out),
                              args.steps, args.warmup)
    _log("batching: buckets one by one")

    def per_bucket(t):
        for i in range(len(buckets)):
            t(f"bucket{i}", plan.forward_bucket, i, obs, out, True)
    _, bms = timed_steps(torch, per_bucket, args.steps, args.warmup)
    bucket_ms = [bms[f"bucket{i}"] for i in range(len(buckets))]
    dom = int(np.argmax(bucket_ms))
    achieved = bucket_bytes[dom] / (bucket_ms[dom] * 1e-3) / 1e9
    eng = {1: "lds", 2: "register"}
    kern = ("forward_rf_queue_kernel" if buckets[dom]["engine"] == 2
            else "forward_queue_kernel")
    traffic = recorded_traffic(eng[buckets[dom]["engine"]], buckets[dom]["obs_per_lane"],
                               buckets[dom]["rows_class"])
    roofline = {"bound": "hbm", "kernel": f"{kern} (bucket {dom}: "
                f"{eng[buckets[dom]['engine']]} engine, {buckets[dom]['obs_per_lane']} obs per "
                f"lane, rows <= {buckets[dom]['rows_class']})",
                "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                "algorithmic_bytes": bucket_bytes[dom], "avg_ms": bucket_ms[dom]}
    passes = pop.P * B
    info = {
        "workload": "batching: 10000 genomes, hidden nodes log-uniform 10..500, "
                    "connections 2-4x hidden (max 2000), 27 -> 8, ragged layout, 256 N(0,1) "
                    "observations per genome; step = batched forward by a tuned plan "
                    "(persistent bucket kernels in one hipGraph)",
        "population": pop.P, "obs_per_genome": B, "n_in": I, "n_out": O,
        "mean_nodes": float(nv.mean()), "mean_enabled_edges": float(ne.mean()),
    }
    res = {
        "passes": passes, "ms_per_step": graph_ms, "roofline": roofline, "config": info,
        "whole_step_hbm_frac": total_bytes / (graph_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "algorithmic_bytes_per_step": total_bytes,
        "plain_per_bucket": {"value": passes / (plain_ms * 1e-3), "ms_per_step": plain_ms,
                             "persistent_graph_speedup": plain_ms / graph_ms},
        "buckets": [{**b, "ms_alone": m, "algorithmic_bytes": by}
                    for b, m, by in zip(buckets, bucket_ms, bucket_bytes)],
    }
    return res, pop, obs_np


def recorded_traffic(engine, obs_per_lane, rows_class):
    """HBM bytes per launch of a bucket kernel from a committed rocprofv3 summary
    (FETCH_SIZE + WRITE_SIZE, copy-calibrated), if one matches this bucket and
    the kernel's sources are unchanged since it was taken; else None."""
    import glob
    import hashlib
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.txt"))):
        text = open(path).read()
        if "```json" not in text:
            continue
        rec = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
        if (rec.get("workload"), rec.get("engine"), rec.get("obs_per_lane"),
                rec.get("rows_class")) != ("batching", engine, obs_per_lane, rows_class):
            continue
        h = hashlib.sha256()
        for src in rec["sources"]:
            with open(os.path.join(ROOT, src), "rb") as f:
                h.update(f.read())
        if h.hexdigest() == rec["sources_sha256"]:
            return rec["traffic_bytes_per_launch"]
    return None


def bucket_members(pop, tr, buckets):
    """Genome indices of each bucket, by the plan's documented rule: register
    buckets by prog_rows (flagged genomes in the first), LDS buckets by n_rows
    for the programs too large for the largest register file."""
    import numpy as np
    st = tr.status.cpu().numpy()[:pop.P]
    pr = tr.prog_rows.cpu().numpy()[:pop.P]
    nr = tr.n_rows.cpu().numpy()[:pop.P]
    reg_max = max(b["rows_class"] for b in buckets if b["engine"] == 2)
    lists, lo_reg, lo_lds = [], 0, None
    for b in buckets:
        if b["engine"] == 2:
            m = (st == 0) & (pr > lo_reg) & (pr <= b["rows_class"])
            if lo_reg == 0:
                m |= st != 0
            lo_reg = b["rows_class"]
        else:
            m = (st == 0) & (pr > reg_max) & (nr <= b["rows_class"])
            if lo_lds is not None:
                m &= nr > lo_lds
            lo_lds = b["rows_class"]
        lists.append(np.flatnonzero(m))
    return lists


def cpu_baseline_forward(pop, obs, budget_s, label):
    """The oracle as it stands, one process: transform + forward of a sample of
    genomes with all their observations, scaled to passes per second."""
    import numpy as np
    import oracle
    rng = np.random.default_rng(0)
    order = rng.permutation(pop.P)
    t0 = time.perf_counter()
    n_g = 0
    while time.perf_counter() - t0 < budget_s and n_g < pop.P:
        g = int(order[n_g])
        gen = oracle.decode(pop, g)
        oracle.forward(gen, oracle.transform(gen), obs[g])
        n_g += 1
    sec = time.perf_counter() - t0
    B = obs.shape[1]
    return {"value": n_g * B / sec, "unit": "genome-forward-passes/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{n_g} random genomes of the {label} population x all {B} observations "
                      f"each (decode + transform + forward), float64 NumPy, one process, "
                      f"{sec:.1f} s"}


# ------------------------------------------------------------------- control

def control(torch, tn, synth, args):
    import numpy as np
    pop = synth.control_population()
    B = 1000
    obs_np = synth.normal_obs(pop.P, B, pop.n_in, synth.CONFIG_SEEDS["control"] + 100)
    dp = device_population(torch, tn, pop)
    obs = torch.from_numpy(obs_np).cuda()
    tr = tn.Transformed(dp)
    out = torch.empty((pop.P, B, pop.n_out), dtype=torch.float32, device="cuda")
    ws = tn.DistanceWorkspace(dp)
    dist = (torch.empty((pop.P, pop.P), dtype=torch.float32, device="cuda"),
            torch.empty((pop.P, pop.P), dtype=torch.int32, device="cuda"),
            torch.empty((pop.P, pop.P), dtype=torch.int32, device="cuda"))
    tn.transform(dp, out=tr)

    def step(t):
        t("transform", tn.transform, dp, out=tr)
        t("forward", tn.forward, dp, tr, obs, out=out)
        t("distance", tn.distance, dp, workspace=ws, out=dist)
    step_ms, ms = timed_steps(torch, step, args.steps, args.warmup)
    nv, ne = genome_sizes(torch, pop, tr)
    I, O = pop.n_in, pop.n_out
    fwd_bytes = (4 * pop.P * B * (I + O) + int(np.sum(4 * (nv + 1) + 20 * nv + 8 * ne))
                 + 4 * pop.P * (I + O) + 8 * pop.P)
    achieved = fwd_bytes / (ms["forward"] * 1e-3) / 1e9
    return {
        "workload": "control-policy: 1000 genomes, 17 -> 6, N_max 64, C_max 256, 1000 N(0,1) "
                    "observations per genome; step = transform + forward (the library's "
                    "engine choice: register engine, four tiles of 64 observations per "
                    "wavefront) + 1000 x 1000 compatibility distance",
        "value": pop.P * B / (step_ms * 1e-3), "unit": "genome-forward-passes/s",
        "ms_per_step": step_ms, "call_ms": ms,
        "forward_roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                             "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                             "algorithmic_bytes": fwd_bytes},
        "distance_pairs_per_s": pop.P * pop.P / (ms["distance"] * 1e-3),
    }


# ----------------------------------------------------------- differentiation

def differentiation(torch, tn, synth, args):
    import numpy as np
    pop = synth.differentiation_population()
    X = synth.uniform_inputs(1024, 4, synth.CONFIG_SEEDS["differentiation"] + 100)
    T = synth.target_mlp(X, 32, 2, synth.CONFIG_SEEDS["differentiation"] + 200)
    dp = device_population(torch, tn, pop)
    tr = tn.transform(dp)
    Xt, Tt = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
    step_ms, ms = timed_steps(
        torch, lambda t: t("forward_backward_mse", tn.forward_backward_mse, dp, tr, Xt, Tt),
        args.steps, args.warmup)
    nv, ne = genome_sizes(torch, pop, tr)
    # gradients written + program read twice (forward and reverse sweep) + data
    by = int(4 * pop.P * (pop.C_max + pop.N_max) + 2 * np.sum(24 * nv + 8 * ne)
             + X.nbytes + T.nbytes)
    achieved = by / (ms["forward_backward_mse"] * 1e-3) / 1e9
    return {
        "workload": "differentiation: 4096 genomes 4 -> 2 (N_max 64, C_max 256), 1024 shared "
                    "U(-1,1) samples, MSE against a fixed 4-32-2 tanh MLP; step = forward + "
                    "adjoint (dL/dW, dL/db)",
        "value": pop.P * 1024 / (step_ms * 1e-3), "unit": "sample-passes/s (forward+adjoint)",
        "ms_per_step": step_ms, "roofline": {"bound": "hbm", "achieved": achieved,
                                             "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                             "frac": achieved / HBM_PEAK_GBS,
                                             "algorithmic_bytes": by},
    }


# ------------------------------------------------------------------ hyperneat

def hyperneat(torch, tn, synth, args):
    pop = synth.cppn_population()
    dp = device_population(torch, tn, pop)
    tr = tn.transform(dp)
    grid, n_out, B = 32, 8, 128
    S = grid * grid
    g = torch.Generator().manual_seed(synth.CONFIG_SEEDS["cppn"] + 100)
    xb = torch.randn((pop.P, B, S), generator=g).to(torch.bfloat16).cuda()
    dy = torch.randn((pop.P, B, n_out), generator=g).cuda()
    state = {}

    def step(t):
        w1t, w2t = t("cppn_query", tn.cppn_query, dp, tr, grid, n_out, 0.2)
        h, y = t("substrate_forward", tn.substrate_forward, w1t, w2t, xb, grid, n_out)
        dw1t, dw2t = t("substrate_backward", tn.substrate_backward, w2t, xb, h, dy, grid, n_out)
        t("cppn_backward", tn.cppn_backward, dp, tr, dw1t, dw2t, grid, n_out)
        state["w"] = (w1t, w2t)
    steps = max(2, args.steps // 4)
    step_ms, ms = timed_steps(torch, step, steps, 1)
    flops = 2.0 * pop.P * B * S * S + 2.0 * pop.P * B * S * n_out
    w_bytes = 2 * pop.P * (S * S + S * n_out)
    fwd_bytes = w_bytes + xb.numel() * 2 + 4 * pop.P * B * (S + n_out)
    return {
        "workload": "hyperneat: 1000 CPPNs 5 -> 1 (N_max 32, C_max 96) queried on a 32x32 / "
                    "32x32 / 8 grid substrate (1,056,768 queries each), |w| < 0.2 -> 0, bf16; "
                    "128 N(0,1) bf16 inputs per genome; step = query + substrate forward + "
                    "substrate backward + CPPN adjoint",
        "ms_per_step": step_ms, "call_ms": ms, "steps": steps,
        "queries_per_s": pop.P * (S * S + S * n_out) / (ms["cppn_query"] * 1e-3),
        "substrate_forward": {
            "tflops": flops / (ms["substrate_forward"] * 1e-3) / 1e12,
            "mfma_frac": flops / (ms["substrate_forward"] * 1e-3) / 1e12 / BF16_PEAK_TFLOPS,
            "hbm_frac": fwd_bytes / (ms["substrate_forward"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "algorithmic_bytes": fwd_bytes},
    }


def main():
    args = _args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              f"(asked for --gpus {args.gpus}, WORLD_SIZE {world}).", file=sys.stderr)
        sys.exit(2)
    import torch
    import synth
    import paper_2504_08339_amd as tn
    assert torch.cuda.is_available(), "bench.py needs a GPU"

    _log("building the batching workload")
    head, pop, obs_np = batching(torch, tn, synth, args)
    others = {}
    if not args.only_headline:
        for name, fn in (("control", control), ("differentiation", differentiation),
                         ("hyperneat", hyperneat)):
            _log(f"workload {name}")
            others[name] = fn(torch, tn, synth, args)
            torch.cuda.empty_cache()
    if args.copy_calibration:
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
    cpu = None
    if not args.no_cpu_baseline:
        _log("timing the CPU oracle sample")
        cpu = cpu_baseline_forward(pop, obs_np, args.cpu_seconds, "batching")

    line = {
        "metric": METRIC, "value": head["passes"] / (head["ms_per_step"] * 1e-3),
        "unit": "genome-forward-passes/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": head["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": head["config"], "roofline": head["roofline"], "cpu_baseline": cpu,
        "plain_per_bucket": head["plain_per_bucket"],
        "whole_step_hbm_frac": head["whole_step_hbm_frac"],
        "algorithmic_bytes_per_step": head["algorithmic_bytes_per_step"],
        "buckets": head["buckets"], "workloads": others,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
