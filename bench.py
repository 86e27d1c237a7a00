#!/usr/bin/env python3
"""Throughput of the population-evaluation hot path on one MI355X.

Prints ONE JSON line. A step is one pass of the hot path over one batch of
synthetic input, with every input already resident in device memory:

  control  (default) 1000 genomes, 17 -> 6, N_max 64, C_max 256, 1000 N(0,1)
           observations per genome: transform + forward (1e6 genome-forward
           passes) + the 1000 x 1000 compatibility distance matrix.

`value` is genome-forward passes per second over the timed steps (P * B per
step / time per step). Each library call is bracketed by HIP events on the
stream it runs on; the dominant call's average duration gives the roofline
figure. The CPU oracle is timed on a bounded sample for `cpu_baseline`.
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


def _args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="control", choices=["control"])
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="rough budget of the CPU-oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one 1 GiB device copy (counter calibration under rocprofv3)")
    return ap.parse_args()


class CallTimer:
    """HIP events around each library call, on torch's current stream (the stream
    every call is launched on)."""

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

    def reset(self):
        self.pairs = {}

    def mean_ms(self):
        return {n: sum(a.elapsed_time(b) for a, b in v) / len(v) for n, v in self.pairs.items()}


def control_workload(torch, tn, synth):
    import numpy as np
    pop = synth.control_population()
    B = 1000
    obs_np = synth.normal_obs(pop.P, B, pop.n_in, synth.CONFIG_SEEDS["control"] + 100)
    arrays = {k: getattr(pop, k) for k in ("node_key", "node_bias", "node_resp", "node_act",
                                           "node_agg", "conn_in", "conn_out", "conn_w", "conn_en")}
    dp = tn.Population.from_numpy(pop.n_in, pop.n_out, pop.N_max, pop.C_max, arrays, device="cuda")
    obs = torch.from_numpy(obs_np).cuda()
    tr = tn.Transformed(dp)
    out = torch.empty((pop.P, B, pop.n_out), dtype=torch.float32, device="cuda")
    ws = tn.DistanceWorkspace(dp)
    dist = (torch.empty((pop.P, pop.P), dtype=torch.float32, device="cuda"),
            torch.empty((pop.P, pop.P), dtype=torch.int32, device="cuda"),
            torch.empty((pop.P, pop.P), dtype=torch.int32, device="cuda"))

    def step(timer):
        timer("transform", tn.transform, dp, out=tr)
        timer("forward", tn.forward, dp, tr, obs, out=out)
        timer("distance", tn.distance, dp, workspace=ws, out=dist)

    # algorithmic bytes, counted from the actual population
    tn.transform(dp, out=tr)
    torch.cuda.synchronize()
    nv = tr.n_valid.cpu().numpy().astype(np.int64)
    rp = tr.row_ptr.cpu().numpy().reshape(pop.P, pop.N_max + 1)
    ne = rp[np.arange(pop.P), nv].astype(np.int64)
    I, O = pop.n_in, pop.n_out
    fwd_bytes = (4 * pop.P * B * I + 4 * pop.P * B * O          # observations in, outputs out
                 + int(np.sum(4 * (nv + 1) + 12 * nv + 8 * ne))  # row_ptr, fn/bias/resp, edges
                 + 4 * pop.P * (I + O) + 8 * pop.P)              # io positions, status/n_valid
    valid_rows = pop.nbytes_valid()
    tr_bytes = valid_rows + int(np.sum(20 * nv + 4 * (nv + 1) + 12 * ne)) + 4 * pop.P * (I + O + 2)
    info = {
        "workload": "control-policy: 1000 genomes, 17 inputs -> 6 outputs, N_max 64, C_max 256, "
                    "1000 N(0,1) observations per genome; step = transform + forward + "
                    "1000x1000 compatibility distance",
        "population": pop.P, "obs_per_genome": B, "n_in": I, "n_out": O, "N_max": pop.N_max,
        "C_max": pop.C_max, "mean_nodes": float(nv.mean()), "mean_enabled_edges": float(ne.mean()),
    }
    bytes_per_call = {"forward": fwd_bytes, "transform": tr_bytes}
    return pop, obs_np, step, pop.P * B, info, bytes_per_call


def cpu_baseline_control(pop, obs, budget_s):
    """The oracle as it stands, single process: transform + forward of a sample of
    genomes (all their observations) and distances of a sample of pairs, each
    scaled to the whole step."""
    import numpy as np
    import oracle
    rng = np.random.default_rng(0)
    t0 = time.perf_counter()
    n_g = 0
    order = rng.permutation(pop.P)
    while time.perf_counter() - t0 < 0.5 * budget_s and n_g < pop.P:
        g = int(order[n_g])
        gen = oracle.decode(pop, g)
        oracle.forward(gen, oracle.transform(gen), obs[g])
        n_g += 1
    t_fwd = (time.perf_counter() - t0) / n_g
    genes = {}
    t1 = time.perf_counter()
    n_p = 0
    while time.perf_counter() - t1 < 0.5 * budget_s:
        i, j = (int(x) for x in rng.integers(0, pop.P, 2))
        for k in (i, j):
            if k not in genes:
                genes[k] = oracle.genome_genes(pop, k)
        oracle.distance(genes[i], genes[j])
        n_p += 1
    t_pair = (time.perf_counter() - t1) / n_p
    step_s = t_fwd * pop.P + t_pair * pop.P * pop.P
    B = obs.shape[1]
    return {"value": pop.P * B / step_s, "unit": "genome-forward-passes/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{n_g} genomes x {B} observations (transform + forward) and {n_p} "
                      f"genome pairs (distance), float64 NumPy / Python, one process; "
                      f"scaled to 1000 genomes + 1e6 pairs per step",
            "seconds_per_step": step_s}


def main():
    args = _args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              f"(asked for --gpus {args.gpus}, WORLD_SIZE {world}).", file=sys.stderr)
        sys.exit(2)
    import torch
    import synth
    import paper_2504_08339_amd as tn
    assert torch.cuda.is_available(), "bench.py needs a GPU"

    print("bench: building the control workload", file=sys.stderr, flush=True)
    pop, obs_np, step, passes, info, bytes_per_call = control_workload(torch, tn, synth)
    print("bench: timing", file=sys.stderr, flush=True)
    timer = CallTimer(torch)
    for _ in range(args.warmup):
        step(timer)
    torch.cuda.synchronize()
    timer.reset()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(timer)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = timer.mean_ms()
    step_ms = 1e3 * wall / args.steps

    dominant = max(ms, key=ms.get)
    roof_kernel = dominant if dominant in bytes_per_call else "forward"
    achieved = bytes_per_call[roof_kernel] / (ms[roof_kernel] * 1e-3) / 1e9
    roofline = {"bound": "hbm", "kernel": roof_kernel, "achieved": achieved,
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                "traffic": None, "algorithmic_bytes": bytes_per_call[roof_kernel],
                "avg_ms": ms[roof_kernel]}
    if args.copy_calibration:
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()

    cpu = None
    if not args.no_cpu_baseline:
        print("bench: timing the CPU oracle sample", file=sys.stderr, flush=True)
        cpu = cpu_baseline_control(pop, obs_np, args.cpu_seconds)

    line = {
        "metric": METRIC, "value": passes / (step_ms * 1e-3), "unit": "genome-forward-passes/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": step_ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic", "config": info, "kernel_ms": ms, "dominant_call": dominant,
        "roofline": roofline, "cpu_baseline": cpu,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
