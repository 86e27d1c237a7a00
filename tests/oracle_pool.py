"""Oracle references over whole workloads, in parallel worker processes (test
infrastructure: the oracle is the plain float64 definition and slow).

Every worker rebuilds the seeded workload itself (the generators are
deterministic), so only genome index ranges and results cross the process
boundary. Workers are started with "spawn" and import only numpy, the oracle
and the input generators: they never touch the GPU.
"""
import concurrent.futures as cf
import multiprocessing as mp
import os

import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

_CACHE = {}
RECURRENT_B = 1000      # observations per genome of the recurrent workload
RECURRENT_T = 10        # sweeps of the recurrent workload


def _workload(name):
    if name in _CACHE:
        return _CACHE[name]
    import synth
    s = synth.CONFIG_SEEDS
    if name == "control":
        pop = synth.control_population()
        data = (synth.normal_obs(pop.P, 1000, pop.n_in, s["control"] + 100),)
    elif name == "batching":
        pop = synth.batching_population()
        data = (synth.normal_obs(pop.P, 256, pop.n_in, s["batching"] + 100),)
    elif name == "differentiation":
        pop = synth.differentiation_population()
        X = synth.uniform_inputs(1024, 4, s["differentiation"] + 100)
        data = (X, synth.target_mlp(X, 32, 2, s["differentiation"] + 200))
    elif name == "recurrent":
        pop = synth.recurrent_population()
        data = (synth.normal_obs(pop.P, RECURRENT_B, pop.n_in, s["recurrent"] + 100),)
    else:
        raise ValueError(name)
    _CACHE[name] = (pop, data)
    return _CACHE[name]


def _forward_chunk(args):
    name, lo, hi = args
    import oracle
    pop, (obs,) = _workload(name)
    ys, cs, st = [], [], []
    for g in range(lo, hi):
        gen = oracle.decode(pop, g)
        tr = oracle.transform(gen)
        y, c = oracle.forward(gen, tr, obs[g], with_cond=True)
        ys.append(y)
        cs.append(c)
        st.append(tr.status)
    return lo, np.stack(ys), np.stack(cs), np.array(st)


def _recurrent_chunk(args):
    name, lo, hi = args
    import oracle
    pop, (obs,) = _workload(name)
    Y, C, st = oracle.recurrent_population(pop, obs, RECURRENT_T, genomes=range(lo, hi),
                                           with_cond=True)
    return lo, Y, C, st


def _grad_chunk(args):
    name, lo, hi = args
    import oracle
    pop, (X, T) = _workload(name)
    loss = np.zeros(hi - lo)
    dW = np.zeros((hi - lo, pop.C_max))
    db = np.zeros((hi - lo, pop.N_max))
    st = np.zeros(hi - lo, np.int64)
    for a, g in enumerate(range(lo, hi)):
        gen = oracle.decode(pop, g)
        tr = oracle.transform(gen)
        st[a] = tr.status
        Y = oracle.forward(gen, tr, X)
        w, b = oracle.backward(gen, tr, X, 2.0 * (Y - T) / Y.size)
        loss[a] = float(np.mean((Y - T) ** 2))
        for r, v in w.items():
            dW[a, r] = v
        for r, v in b.items():
            db[a, r] = v
    return lo, loss, dW, db, st


def workers():
    # the GPU machine gives one GPU's share of 16 host cores, whatever the machine shows
    return max(1, min(16, len(os.sched_getaffinity(0))))


def _run(fn, name, P, chunk):
    ranges = [(name, lo, min(P, lo + chunk)) for lo in range(0, P, chunk)]
    ctx = mp.get_context("spawn")
    with cf.ProcessPoolExecutor(workers(), mp_context=ctx) as ex:
        return sorted(ex.map(fn, ranges), key=lambda r: r[0])


def forward_reference(name, P, chunk=250):
    """(Y [P][B][O], cond [P][B][O], status [P]) of the named workload."""
    parts = _run(_forward_chunk, name, P, chunk)
    return (np.concatenate([p[1] for p in parts]), np.concatenate([p[2] for p in parts]),
            np.concatenate([p[3] for p in parts]))


def recurrent_reference(P, chunk=50):
    """(Y [P][B][O], cond, status [P]) of the recurrent workload after
    RECURRENT_T sweeps."""
    parts = _run(_recurrent_chunk, "recurrent", P, chunk)
    return (np.concatenate([p[1] for p in parts]), np.concatenate([p[2] for p in parts]),
            np.concatenate([p[3] for p in parts]))


def mse_grad_reference(name, P, chunk=256):
    """(loss [P], dW [P][C_max], db [P][N_max], status [P]) of the MSE workload."""
    parts = _run(_grad_chunk, name, P, chunk)
    return tuple(np.concatenate([p[i] for p in parts]) for i in range(1, 5))
