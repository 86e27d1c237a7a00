"""One generation of NEAT on a padded population (Algorithm 1's loop body:
divide the population into species by distance, decide how many children each
species gets from the fitness, and make them by crossover and mutation), plus
the initial population (Algorithm 1's first step). Hyperparameters are those
of Appendix A (values of Appendix C by default).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper names these steps and their hyperparameters but not their rules.
Readings taken here (each step plain and in order):

Initial population. Every genome holds the input nodes (keys 0..I-1) and the
output nodes (keys I..I+O-1) in its first node rows and every input -> output
connection, enabled, in row i*O + o. Each node row's bias and response and
each connection's weight come from their initial distributions (mean + std *
z with the normals of the mutation layout: Z[4 + 2r + k] for node row r, Z[4
+ 2 N_max + r] for connection row r), activation and aggregation the defaults.

Species table. Up to max_species slots, each alive or free, with a
representative genome (its rows), the best species fitness so far, the
generation of its last improvement and its size (children given) in the last
generation.

1. Speciation. The distance is the node-inclusive one (``compat``) with the
   paper's coefficient pair, evaluated in float32 in ascending key order (the
   precision in which the kernel takes the threshold decisions; ``distance_f32``).
   a) Every genome joins the alive species whose representative is nearest,
      if that distance is below compatibility_threshold (ties: lowest slot).
   b) The others, in ascending genome index: while free slots remain, a
      genome joins the nearest species founded in this step before it if one
      is below the threshold (ties: lowest slot), else founds a species in the
      lowest free slot (itself its representative for the rest of the step).
      With no free slot left, it joins the nearest alive species, old or new,
      whatever the distance (ties: lowest slot; a NaN distance, from a genome
      without a gene set, counts as infinite).
   c) An old species that got no member is dropped.
2. Species fitness is the largest member fitness. It improves when above the
   best so far (which it then becomes, with the generation). A species is
   stagnant when generation - last improvement >= max_stagnation, except the
   species_elitism species of largest fitness (ties: lowest slot). Stagnant
   species get no children and are dropped.
3. Children per surviving species (float32, in slot order):
     lo, hi = smallest and largest member fitness over surviving species;
     af_s = (mean member fitness - lo) / max(hi - lo, 1), the mean summed in
            ascending genome order;
     target_s = P * af_s / sum af (P / n_species when sum af is 0);
     spawn_s = prev_size_s + (target_s - prev_size_s) * spawn_number_change_rate;
     share_s = spawn_s * P / sum spawn (P / n_species when sum spawn is 0);
     count_s = floor(share_s), then one more for the P - sum count species of
     largest share_s - count_s (ties: lowest slot).
4. Parents. Members of a species are ranked by fitness (largest first; ties:
   lower genome index). The children of the species, in slot order of species
   and then rank order, are first its elites: ranks 0 .. min(genome_elitism,
   count, members) - 1 copied unchanged (second parent -1); then the others
   from two uniform picks among the survivors, ranks 0 .. max(1,
   ceil(survival_threshold * members)) - 1 (product in float32): the fitter
   of the two (ties: lower index) is the first parent.
5. Reproduction of the parent pairs (``reproduce``) with its own draws.
6. Table for the next generation: every surviving species with children keeps
   its slot with its rank-0 member as representative and its count as size;
   the others are freed.

Random numbers are inputs: selection uniforms S [P][2] (the two picks of
child c), and the reproduction draws U, Z of ``reproduce``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np

from . import reproduce as rp
f32 = np.float32


@dataclasses.dataclass
class NeatParams:
    compatibility_threshold: float = 3.5
    compatibility_disjoint: float = 1.0
    compatibility_homologous: float = 0.5
    max_species: int = 10
    species_elitism: int = 2
    max_stagnation: int = 15
    genome_elitism: int = 2
    survival_threshold: float = 0.2
    spawn_number_change_rate: float = 0.5
    mutation: rp.MutationParams = dataclasses.field(default_factory=rp.MutationParams)


@dataclasses.dataclass
class SpeciesTable:
    """Slots of the species table; reps holds one genome's rows per slot."""
    alive: np.ndarray          # [S] bool
    best: np.ndarray           # [S] float32 (-inf for a new species)
    last: np.ndarray           # [S] int
    size: np.ndarray           # [S] int
    reps: List[Optional[rp.Rows]]

    @classmethod
    def empty(cls, S: int) -> "SpeciesTable":
        return cls(np.zeros(S, bool), np.full(S, -np.inf, np.float32), np.zeros(S, np.int64),
                   np.zeros(S, np.int64), [None] * S)


def init_population(P: int, n_in: int, n_out: int, N_max: int, C_max: int, Z: np.ndarray,
                    prm: rp.MutationParams) -> dict:
    """Initial genomes (module docstring), arrays named as in the library."""
    arrays = {
        "node_key": np.full((P, N_max), -1, np.int32),
        "node_bias": np.zeros((P, N_max), np.float32),
        "node_resp": np.zeros((P, N_max), np.float32),
        "node_act": np.zeros((P, N_max), np.uint8),
        "node_agg": np.zeros((P, N_max), np.uint8),
        "conn_in": np.full((P, C_max), -1, np.int32),
        "conn_out": np.full((P, C_max), -1, np.int32),
        "conn_w": np.zeros((P, C_max), np.float32),
        "conn_en": np.zeros((P, C_max), np.uint8),
    }
    for g in range(P):
        z = Z[g]
        for r in range(n_in + n_out):
            arrays["node_key"][g, r] = r
            arrays["node_bias"][g, r] = f32(f32(prm.bias_init_mean) +
                                            f32(f32(prm.bias_init_std) * f32(z[4 + 2 * r])))
            arrays["node_resp"][g, r] = f32(f32(prm.resp_init_mean) +
                                            f32(f32(prm.resp_init_std) * f32(z[4 + 2 * r + 1])))
            arrays["node_act"][g, r] = prm.act_default
            arrays["node_agg"][g, r] = prm.agg_default
        for i in range(n_in):
            for o in range(n_out):
                r = i * n_out + o
                arrays["conn_in"][g, r] = i
                arrays["conn_out"][g, r] = n_in + o
                arrays["conn_w"][g, r] = f32(f32(prm.weight_init_mean) + f32(
                    f32(prm.weight_init_std) * f32(z[4 + 2 * N_max + r])))
                arrays["conn_en"][g, r] = 1
    return arrays


def _genes_of_rows(rows: rp.Rows, n_in: int):
    """node_genes() of one genome's rows: (nodes, conns) dicts or None."""
    nodes, conns, seen = {}, {}, set()
    for r in range(rows.key.shape[0]):
        k = int(rows.key[r])
        if k < 0:
            continue
        if k in seen:
            return None
        seen.add(k)
        if k >= n_in:
            nodes[k] = (f32(rows.bias[r]), f32(rows.resp[r]), int(rows.act[r]), int(rows.agg[r]))
    for r in range(rows.cin.shape[0]):
        a, b = int(rows.cin[r]), int(rows.cout[r])
        if a < 0 or b < 0:
            continue
        if (a, b) in conns:
            return None
        conns[(a, b)] = (f32(rows.w[r]), f32(0.0), int(bool(rows.en[r])), 0)
    return nodes, conns


def distance_f32(a, b, c_d: float, c_h: float) -> np.float32:
    """The node-inclusive distance of ``compat`` with every operation rounded
    to float32: per shared gene the term ((|da0| + |da1|) + [c0 differ]) + [c1
    differ], summed in ascending key order; per gene kind (c_d * D + c_h * H) /
    max(n1, n2), products and sum rounded separately; node part + connection
    part. NaN when either genome has no gene set."""
    if a is None or b is None:
        return f32(np.nan)
    total = f32(0.0)
    for x, y in ((a[0], b[0]), (a[1], b[1])):
        kx, ky = set(x), set(y)
        hom = sorted(kx & ky)
        d = len(kx) + len(ky) - 2 * len(hom)
        n = max(len(kx), len(ky))
        if n == 0:
            continue
        H = f32(0.0)
        for k in hom:
            p, q = x[k], y[k]
            t = f32(f32(abs(f32(p[0] - q[0]))) + f32(abs(f32(p[1] - q[1]))))
            t = f32(t + f32(1.0 if p[2] != q[2] else 0.0))
            t = f32(t + f32(1.0 if p[3] != q[3] else 0.0))
            H = f32(H + t)
        num = f32(f32(f32(c_d) * f32(d)) + f32(f32(c_h) * H))
        total = f32(total + f32(num / f32(n)))
    return total


def speciate(pop, table: SpeciesTable, prm: NeatParams) -> Tuple[np.ndarray, List[int]]:
    """Step 1: species slot of every genome; also the list of slots founded."""
    P, S = pop.P, len(table.alive)
    thr = f32(prm.compatibility_threshold)
    genes = [_genes_of_rows(rp.Rows.of(pop, g), pop.n_in) for g in range(P)]
    rep_genes = [None if not table.alive[s] else _genes_of_rows(table.reps[s], pop.n_in)
                 for s in range(S)]

    def dist(g, other):
        return distance_f32(genes[g], other, prm.compatibility_disjoint,
                            prm.compatibility_homologous)

    sp = np.full(P, -1, np.int64)
    for g in range(P):
        best, bd = -1, None
        for s in range(S):
            if not table.alive[s]:
                continue
            d = dist(g, rep_genes[s])
            if d < thr and (bd is None or d < bd):
                best, bd = s, d
        sp[g] = best
    alive = table.alive.copy()
    founded: List[int] = []
    founder_genes = {}
    for g in range(P):
        if sp[g] >= 0:
            continue
        free = [s for s in range(S) if not alive[s]]
        if free:
            best, bd = -1, None
            for s in founded:
                d = dist(g, founder_genes[s])
                if d < thr and (bd is None or d < bd):
                    best, bd = s, d
            if best >= 0:
                sp[g] = best
                continue
            s = free[0]
            alive[s] = True
            founded.append(s)
            founder_genes[s] = genes[g]
            sp[g] = s
        else:
            best, bd = -1, None
            for s in range(S):
                if not alive[s]:
                    continue
                other = founder_genes[s] if s in founder_genes else rep_genes[s]
                d = dist(g, other)
                d = f32(np.inf) if np.isnan(d) else d   # NaN: no gene set, farthest
                if bd is None or d < bd:
                    best, bd = s, d
            sp[g] = best
    return sp, founded


def rank_members(fit: np.ndarray, sp: np.ndarray):
    """Per genome its rank in its species (largest fitness first, ties lower
    index), and per slot the members in rank order."""
    P = len(fit)
    members = {}
    for g in range(P):
        members.setdefault(int(sp[g]), []).append(g)
    order = {}
    rank = np.zeros(P, np.int64)
    for s, ms in members.items():
        ms = sorted(ms, key=lambda g: (-float(f32(fit[g])), g))
        order[s] = ms
        for i, g in enumerate(ms):
            rank[g] = i
    return rank, order


def allocate(fit: np.ndarray, sp: np.ndarray, table: SpeciesTable, founded: List[int],
             generation: int, prm: NeatParams, P: int):
    """Steps 2-3: (counts [S], surviving mask [S], updated best / last)."""
    S = len(table.alive)
    fit = fit.astype(np.float32)
    best = table.best.copy()
    last = table.last.copy()
    size = table.size.copy()
    for s in founded:
        best[s], last[s], size[s] = f32(-np.inf), generation, 0
    present = [s for s in range(S) if np.any(sp == s)]
    sfit = {}
    for s in present:
        sfit[s] = max(f32(fit[g]) for g in range(P) if sp[g] == s)
        if sfit[s] > best[s]:
            best[s], last[s] = sfit[s], generation
    ranked = sorted(present, key=lambda s: (-float(sfit[s]), s))
    protected = set(ranked[:prm.species_elitism])
    surviving = [s for s in present
                 if s in protected or generation - last[s] < prm.max_stagnation]
    counts = np.zeros(S, np.int64)
    if not surviving:
        return counts, np.zeros(S, bool), best, last
    member_fits = [f32(fit[g]) for g in range(P) if sp[g] in surviving]
    lo, hi = min(member_fits), max(member_fits)
    rng = f32(max(f32(hi - lo), f32(1.0)))
    af = {}
    for s in surviving:
        tot, n = f32(0.0), 0
        for g in range(P):
            if sp[g] == s:
                tot = f32(tot + f32(fit[g]))
                n += 1
        mean = f32(tot / f32(n))
        af[s] = f32(f32(mean - lo) / rng)
    af_sum = f32(0.0)
    for s in surviving:
        af_sum = f32(af_sum + af[s])
    ns = f32(len(surviving))
    rate = f32(prm.spawn_number_change_rate)
    spawn = {}
    for s in surviving:
        target = f32(f32(f32(P) * af[s]) / af_sum) if af_sum > 0 else f32(f32(P) / ns)
        prev = f32(size[s])
        spawn[s] = f32(prev + f32(f32(target - prev) * rate))
    sp_sum = f32(0.0)
    for s in surviving:
        sp_sum = f32(sp_sum + spawn[s])
    share = {}
    for s in surviving:
        share[s] = f32(f32(spawn[s] * f32(P)) / sp_sum) if sp_sum > 0 else f32(f32(P) / ns)
        counts[s] = int(math.floor(share[s]))
    left = P - int(counts.sum())
    by_rem = sorted(surviving, key=lambda s: (-float(f32(share[s] - f32(counts[s]))), s))
    for s in by_rem[:left]:
        counts[s] += 1
    surv = np.zeros(S, bool)
    surv[surviving] = True
    return counts, surv, best, last


def select_parents(fit: np.ndarray, order, counts: np.ndarray, sel: np.ndarray,
                   prm: NeatParams) -> np.ndarray:
    """Step 4: parents [P][2] in child order."""
    fit = fit.astype(np.float32)
    out = []
    for s in range(len(counts)):
        c = int(counts[s])
        if c == 0:
            continue
        ms = order[s]
        n = len(ms)
        e = min(prm.genome_elitism, c, n)
        k = max(1, int(math.ceil(f32(f32(prm.survival_threshold) * f32(n)))))
        for i in range(c):
            if i < e:
                out.append((ms[i], -1))
                continue
            cidx = len(out)
            a = ms[rp._pick(sel[cidx, 0], k)]
            b = ms[rp._pick(sel[cidx, 1], k)]
            if (f32(fit[b]) > f32(fit[a])) or (fit[b] == fit[a] and b < a):
                a, b = b, a
            out.append((a, b))
    return np.array(out, np.int64).reshape(-1, 2)


def generation(pop, fit: np.ndarray, table: SpeciesTable, gen: int, prm: NeatParams,
               sel: np.ndarray, U: np.ndarray, Z: np.ndarray, next_key: int):
    """One generation: (children arrays, new table, species of each genome,
    parents [P][2], next unused key)."""
    P = pop.P
    sp, founded = speciate(pop, table, prm)
    counts, surv, best, last = allocate(fit, sp, table, founded, gen, prm, P)
    rank, order = rank_members(fit, sp)
    parents = select_parents(fit, order, counts, sel, prm)
    kids, nxt = rp.reproduce(pop, parents, U, Z, prm.mutation, next_key)
    S = len(table.alive)
    new = SpeciesTable.empty(S)
    for s in range(S):
        if surv[s] and counts[s] > 0:
            new.alive[s] = True
            new.best[s] = best[s]
            new.last[s] = last[s]
            new.size[s] = counts[s]
            new.reps[s] = rp.Rows.of(pop, order[s][0])
    return kids, new, sp, parents, nxt
