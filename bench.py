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
                   CPPN adjoint;
  xor              150 XOR genomes (16 / 32 rows), the four XOR rows: transform +
                   forward with the fused fitness (microseconds per call);
  recurrent        1000 recurrent genomes 17 -> 6 (control population plus back
                   edges), 1000 obs each, 10 synchronous sweeps;
  reproduce        1000 children of the control population (crossover +
                   mutation, Appendix C rates, draws resident on the device);
  distance_nodes   1000 x 1000 node-inclusive compatibility distance;
  neat_xor         one NEAT generation on XOR, 150 genomes: transform + fitness +
                   speciation + offspring counts + parents + reproduction (the
                   draws made on the device by torch inside the step).

`value` is genome-forward passes per second (P * B per step / time per step).
The roofline object is for the dominant kernel of the headline step: every
bucket's persistent kernel is also launched alone, bracketed by HIP events on
the stream it runs on, and the slowest one's algorithmic bytes (observations
read, outputs written and the program words its genomes read, counted from
the actual population) over its average duration give `achieved`. Beside the HBM
roofline, a vector-ALU one: lane-operations per forward pass counted from the
actual programs (one fused multiply-add per enabled in-edge, one for z and the
activation's instructions per non-input node) over the non-packed float32 peak
of 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3e12 lane-operations/s; the
larger of the two fractions names the binding roof. The CPU oracle is timed on
a bounded sample, fanned out over the host cores, for `cpu_baseline`.
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
VALU_PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9   # non-packed float32 lane-ops/s
# vector instructions of each activation in the forward engines (act code order:
# identity, sigmoid, tanh, relu, sin, gaussian, abs); tanh evaluates both its
# branches and selects, sin includes the range reduction of sinf
ACT_LANE_OPS = (0, 4, 16, 1, 24, 3, 1)


def lane_ops_per_pass(pop, ne):
    """VALU lane-operations of one forward pass per genome: one FMA per
    enabled in-edge (ne), and per non-input node one FMA for z plus its
    activation's instructions."""
    import numpy as np
    cost = np.array(ACT_LANE_OPS, np.int64)
    out = np.zeros(pop.P, np.int64)
    for g in range(pop.P):
        rows = pop.node_rows(g)
        key, act = rows["key"], rows["act"]
        m = key >= pop.n_in
        out[g] = int(np.sum(1 + cost[np.minimum(act[m], 6)]))
    return out + ne


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


def _roof(bytes_, lane_ops, ms, extra=None):
    """HBM and VALU fractions of one timed kernel; `bound` is the larger."""
    gbs = bytes_ / (ms * 1e-3) / 1e9
    lops = lane_ops / (ms * 1e-3)
    hbm, alu = gbs / HBM_PEAK_GBS, lops / VALU_PEAK_LANE_OPS
    r = {"hbm_achieved_GBs": gbs, "hbm_frac": hbm, "alu_achieved_lane_ops_per_s": lops,
         "alu_frac": alu, "binding": "alu" if alu > hbm else "hbm",
         "algorithmic_bytes": int(bytes_), "lane_ops": int(lane_ops), "avg_ms": ms}
    r.update(extra or {})
    return r


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
    lops = lane_ops_per_pass(pop, ne) * B
    bucket_lops = [int(lops[m].sum()) for m in lists]
    achieved = bucket_bytes[dom] / (bucket_ms[dom] * 1e-3) / 1e9
    alu = bucket_lops[dom] / (bucket_ms[dom] * 1e-3)
    eng = {1: "lds", 2: "register"}
    kern = ("forward_rf_queue_kernel" if buckets[dom]["engine"] == 2
            else "forward_queue_kernel")
    traffic = recorded_traffic(eng[buckets[dom]["engine"]], buckets[dom]["obs_per_lane"],
                               buckets[dom]["rows_class"])
    name = (f"{kern} (bucket {dom}: {eng[buckets[dom]['engine']]} engine, "
            f"{buckets[dom]['obs_per_lane']} obs per lane, rows <= {buckets[dom]['rows_class']})")
    if alu / VALU_PEAK_LANE_OPS > achieved / HBM_PEAK_GBS:
        roofline = {"bound": "alu", "kernel": name, "achieved": alu / 1e12,
                    "peak": VALU_PEAK_LANE_OPS / 1e12, "unit": "T lane-ops/s",
                    "frac": alu / VALU_PEAK_LANE_OPS, "traffic": traffic,
                    "lane_ops": bucket_lops[dom], "hbm_GBs": achieved,
                    "hbm_frac": achieved / HBM_PEAK_GBS,
                    "algorithmic_bytes": bucket_bytes[dom], "avg_ms": bucket_ms[dom]}
    else:
        roofline = {"bound": "hbm", "kernel": name, "achieved": achieved, "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                    "alu_frac": alu / VALU_PEAK_LANE_OPS, "lane_ops": bucket_lops[dom],
                    "algorithmic_bytes": bucket_bytes[dom], "avg_ms": bucket_ms[dom]}
    _log("batching: transform + forward steps")

    def with_transform(t):
        t("transform", tn.transform, dp, out=tr)
        t("graph", plan.forward, obs, out)
    tf_ms, tf_calls = timed_steps(torch, with_transform, args.steps, args.warmup)
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
        "whole_step_alu_frac": int(lops.sum()) / (graph_ms * 1e-3) / VALU_PEAK_LANE_OPS,
        "lane_ops_per_step": int(lops.sum()),
        "transform_plus_forward": {"value": passes / (tf_ms * 1e-3), "ms_per_step": tf_ms,
                                   "transform_ms": tf_calls["transform"]},
        "buckets": [{**b, "ms_alone": m, "algorithmic_bytes": by, "lane_ops": lo,
                     "hbm_frac": by / (m * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "alu_frac": lo / (m * 1e-3) / VALU_PEAK_LANE_OPS}
                    for b, m, by, lo in zip(buckets, bucket_ms, bucket_bytes, bucket_lops)],
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


def _oracle_worker(args):
    """One single-threaded worker: decode + transform + forward of its genomes
    (a ragged subset with their observations) until the time budget runs out;
    returns (genomes done, seconds)."""
    sub, obs, budget_s = args
    import oracle
    t0 = time.perf_counter()
    done = 0
    for g in range(sub.P):
        if time.perf_counter() - t0 >= budget_s:
            break
        gen = oracle.decode(sub, g)
        oracle.forward(gen, oracle.transform(gen), obs[g])
        done += 1
    return done, time.perf_counter() - t0


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline_forward(pop, obs, budget_s, label):
    """The oracle as it stands, fanned out over the host cores this process may
    use (at most 16, the share of one GPU on the box): every worker process
    takes an interleaved slice of a random genome order with all its
    observations and runs until the budget; passes per second = all passes
    done / the slowest worker's time."""
    import concurrent.futures as cf
    import multiprocessing as mp
    import numpy as np
    import synth
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    order = np.random.default_rng(0).permutation(pop.P)
    jobs = []
    for w in range(cores):
        idx = [int(g) for g in order[w::cores]]
        jobs.append((synth.subset(pop, idx), obs[idx], budget_s))
    with cf.ProcessPoolExecutor(cores, mp_context=mp.get_context("spawn")) as ex:
        res = list(ex.map(_oracle_worker, jobs))
    n_g = sum(r[0] for r in res)
    sec = max(r[1] for r in res)
    B = obs.shape[1]
    return {"value": n_g * B / sec, "unit": "genome-forward-passes/s", "cores": cores,
            "kind": "oracle", "cpu_model": _cpu_model(),
            "sample": f"{n_g} random genomes of the {label} population x all {B} observations "
                      f"each (decode + transform + forward), float64 NumPy, {cores} "
                      f"single-threaded worker processes, {sec:.1f} s"}


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
    lops = int(lane_ops_per_pass(pop, ne).sum()) * B
    # distance: each pair walks the column genome's genes once, probing the
    # row genome's hash (about 10 lane-ops per probe: hash load, key compare,
    # branch, count, |dw| and sum), plus the row genome's binary search
    genes = np.array([int(np.sum(pop.conn_rows(g)["in"] >= 0)) for g in range(pop.P)])
    dist_lops = 10 * int(np.sum(genes)) * pop.P // 2 + 10 * pop.P * pop.P // 2
    return {
        "workload": "control-policy: 1000 genomes, 17 -> 6, N_max 64, C_max 256, 1000 N(0,1) "
                    "observations per genome; step = transform + forward (the library's "
                    "engine choice: register engine, four tiles of 64 observations per "
                    "wavefront) + 1000 x 1000 compatibility distance",
        "value": pop.P * B / (step_ms * 1e-3), "unit": "genome-forward-passes/s",
        "ms_per_step": step_ms, "call_ms": ms,
        "forward_roofline": _roof(fwd_bytes, lops, ms["forward"]),
        "distance_pairs_per_s": pop.P * pop.P / (ms["distance"] * 1e-3),
        "distance_roofline": _roof(4 * pop.P * pop.P * 3 + 13 * int(genes.sum()), dist_lops,
                                   ms["distance"]),
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
    # forward lane-ops, then per node act' (about 4) + delta + bias sum, and per
    # edge the dW and upstream-gradient FMAs
    nodes = np.array([int(np.sum(pop.node_rows(g)["key"] >= pop.n_in)) for g in range(pop.P)])
    lops = int((lane_ops_per_pass(pop, ne) + 6 * nodes + 2 * ne).sum()) * 1024
    return {
        "workload": "differentiation: 4096 genomes 4 -> 2 (N_max 64, C_max 256), 1024 shared "
                    "U(-1,1) samples, MSE against a fixed 4-32-2 tanh MLP; step = forward + "
                    "adjoint (dL/dW, dL/db)",
        "value": pop.P * 1024 / (step_ms * 1e-3), "unit": "sample-passes/s (forward+adjoint)",
        "ms_per_step": step_ms, "roofline": _roof(by, lops, ms["forward_backward_mse"]),
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
    import numpy as np
    nv, ne = genome_sizes(torch, pop, tr)
    q = S * S + S * n_out
    # per query: 5 inputs from the query index (about 6 lane-ops) + the CPPN's
    # forward; the adjoint adds its reverse sweep (as the differentiation
    # model) and the threshold test
    fw = lane_ops_per_pass(pop, ne)
    nodes = np.array([int(np.sum(pop.node_rows(g)["key"] >= pop.n_in)) for g in range(pop.P)])
    q_lops = int((fw + 6).sum()) * q
    b_lops = int((2 * fw + 6 * nodes + 2 * ne + 8).sum()) * q
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
        "cppn_query_roofline": _roof(2 * pop.P * q + 4 * pop.P * 16 * 32, q_lops,
                                     ms["cppn_query"]),
        "cppn_backward_roofline": _roof(4 * 2 * pop.P * q, b_lops, ms["cppn_backward"]),
        "substrate_forward": {
            "tflops": flops / (ms["substrate_forward"] * 1e-3) / 1e12,
            "mfma_frac": flops / (ms["substrate_forward"] * 1e-3) / 1e12 / BF16_PEAK_TFLOPS,
            "hbm_frac": fwd_bytes / (ms["substrate_forward"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "algorithmic_bytes": fwd_bytes},
    }


# ------------------------------------------------------------------- xor

def xor(torch, tn, synth, args):
    pop = synth.xor_population()
    dp = device_population(torch, tn, pop)
    X = torch.from_numpy(synth.xor_inputs()).cuda()
    T = torch.from_numpy(synth.xor_targets()).cuda()
    tr = tn.Transformed(dp)

    def step(t):
        t("transform", tn.transform, dp, out=tr)
        t("forward_loss", tn.forward_loss, dp, tr, X, T, -1.0, 4.0, False)
    step_ms, ms = timed_steps(torch, step, max(args.steps, 50), args.warmup)
    return {"workload": "xor: 150 genomes 3 -> 1 (N_max 16, C_max 32), the four XOR rows with "
                        "bias input; step = transform + forward with the fused fitness 4 - SSE",
            "us_per_call": 1e3 * step_ms, "call_us": {k: 1e3 * v for k, v in ms.items()},
            "value": pop.P * 4 / (step_ms * 1e-3), "unit": "genome-forward-passes/s",
            "note": "launch-latency bound (two launches per call); the rooflines say nothing"}


# ------------------------------------------------------------------ recurrent

def recurrent(torch, tn, synth, args):
    import numpy as np
    pop = synth.recurrent_population()
    B, T = 1000, 10
    obs = torch.from_numpy(synth.normal_obs(pop.P, B, pop.n_in,
                                            synth.CONFIG_SEEDS["recurrent"] + 100)).cuda()
    dp = device_population(torch, tn, pop)
    out = torch.empty((pop.P, B, pop.n_out), dtype=torch.float32, device="cuda")
    step_ms, ms = timed_steps(torch, lambda t: t("recurrent", tn.forward_recurrent, dp, obs, T,
                                                 out), args.steps, args.warmup)
    ne = np.array([int(np.sum((pop.conn_rows(g)["in"] >= 0) & (pop.conn_rows(g)["en"] != 0)))
                   for g in range(pop.P)])
    lops = int(lane_ops_per_pass(pop, ne).sum()) * B * T
    by = obs.numel() * 4 + out.numel() * 4 + pop.P * (14 * pop.N_max + 13 * pop.C_max)
    return {"workload": "recurrent: 1000 genomes 17 -> 6 (control population plus up to 12 "
                        "enabled back edges and self-loops each, N_max 64, C_max 256), 1000 "
                        "N(0,1) observations per genome, 10 synchronous sweeps",
            "value": pop.P * B / (step_ms * 1e-3), "unit": "genome-forward-passes/s",
            "ms_per_step": step_ms, "roofline": _roof(by, lops, ms["recurrent"])}


# ------------------------------------------------------------------ reproduce

def reproduce(torch, tn, synth, args):
    import numpy as np
    pop = synth.control_population()
    dp = device_population(torch, tn, pop)
    n = pop.P
    g = torch.Generator(device="cuda").manual_seed(11)
    parents = torch.randint(0, pop.P, (n, 2), device="cuda", generator=g, dtype=torch.int32)
    nu, nz = tn.reproduce_draws(pop.N_max, pop.C_max)
    U = torch.rand((n, nu), device="cuda", generator=g)
    Z = torch.randn((n, nz), device="cuda", generator=g)
    next_key = int(max(pop.node_key.max(), pop.conn_in.max(), pop.conn_out.max())) + 1
    step_ms, ms = timed_steps(torch, lambda t: t("reproduce", tn.reproduce, dp, parents, U, Z,
                                                 None, next_key), args.steps, args.warmup)
    row = 14 * pop.N_max + 13 * pop.C_max
    by = n * (3 * row + 4 * (nu + nz) + 8)   # two parents read, the child written, draws
    return {"workload": "reproduce: 1000 children of the control population (64 / 256 rows), "
                        "random parent pairs, Appendix C rates; step = crossover + mutation "
                        "with resident draws",
            "value": n / (step_ms * 1e-3), "unit": "children/s", "ms_per_step": step_ms,
            "roofline": {"bound": "hbm", "achieved": by / (ms["reproduce"] * 1e-3) / 1e9,
                         "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": by / (ms["reproduce"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                         "algorithmic_bytes": by, "avg_ms": ms["reproduce"]}}


# ------------------------------------------------------------- distance_nodes

def distance_nodes(torch, tn, synth, args):
    pop = synth.control_population()
    dp = device_population(torch, tn, pop)
    out = (torch.empty((pop.P, pop.P), dtype=torch.float32, device="cuda"),
           torch.empty((pop.P, pop.P), dtype=torch.int32, device="cuda"),
           torch.empty((pop.P, pop.P), dtype=torch.int32, device="cuda"))
    step_ms, ms = timed_steps(torch, lambda t: t("distance_nodes", tn.distance_nodes, dp, 1.0,
                                                 0.5, True, out), args.steps, args.warmup)
    return {"workload": "distance_nodes: 1000 x 1000 node-inclusive distance of the control "
                        "population (c_d 1.0, c_h 0.5)",
            "value": pop.P * pop.P / (step_ms * 1e-3), "unit": "pairs/s", "ms_per_step": step_ms}


# ------------------------------------------------------------------- neat_xor

def neat_xor(torch, tn, synth, args):
    P, N, C = 150, 16, 32
    prm = tn.NeatParams(mutation=tn.MutationParams(act_default=1))
    nu, nz = tn.reproduce_draws(N, C)
    g = torch.Generator(device="cuda").manual_seed(5)
    pop, table = tn.neat_init(P, 3, 1, N, C, torch.randn((P, nz), device="cuda", generator=g),
                              prm.mutation, prm.max_species)
    X = torch.from_numpy(synth.xor_inputs()).cuda()
    T = torch.from_numpy(synth.xor_targets()).cuda()
    state = {"pop": pop, "gen": 0, "key": 4, "best": []}

    def step(t):
        p = state["pop"]
        fit, _ = t("fitness", lambda: tn.forward_loss(p, tn.transform(p), X, T, -1.0, 4.0, False))
        sel = torch.rand((P, 2), device="cuda", generator=g)
        U = torch.rand((P, nu), device="cuda", generator=g)
        Z = torch.randn((P, nz), device="cuda", generator=g)
        kids, _, _, nk = t("generation", tn.neat_generation, p, fit, state["gen"], table, sel, U,
                           Z, state["key"], prm)
        state["pop"], state["gen"] = kids, state["gen"] + 1
        state["key"] += 2 * P   # an upper bound of the keys one generation can use
        state["best"].append(fit)
    step_ms, ms = timed_steps(torch, step, max(args.steps, 50), args.warmup)
    best = [float(f.max()) for f in state["best"][-5:]]
    return {"workload": "neat_xor: one NEAT generation on XOR, 150 genomes (16 / 32 rows), "
                        "Appendix C parameters with sigmoid nodes; step = transform + fitness + "
                        "speciation + counts + parents + reproduction (+ device draws)",
            "value": 1e3 / step_ms, "unit": "generations/s", "ms_per_step": step_ms,
            "call_ms": ms, "generations_run": state["gen"], "best_fitness_last": best}


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
                         ("hyperneat", hyperneat), ("xor", xor), ("recurrent", recurrent),
                         ("reproduce", reproduce), ("distance_nodes", distance_nodes),
                         ("neat_xor", neat_xor)):
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
        "whole_step_alu_frac": head["whole_step_alu_frac"],
        "algorithmic_bytes_per_step": head["algorithmic_bytes_per_step"],
        "lane_ops_per_step": head["lane_ops_per_step"],
        "transform_plus_forward": head["transform_plus_forward"],
        "buckets": head["buckets"], "workloads": others,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
