"""Moves synthetic populations to the device and reads results back (tests only)."""
import numpy as np
import torch

import paper_2504_08339_amd as tn

FIELDS = ("node_key", "node_bias", "node_resp", "node_act", "node_agg",
          "conn_in", "conn_out", "conn_w", "conn_en")


def to_device(pop, device="cuda"):
    arrays = {k: getattr(pop, k) for k in FIELDS}
    return tn.Population.from_numpy(pop.n_in, pop.n_out, pop.N_max, pop.C_max, arrays,
                                    device=device, node_off=pop.node_off, conn_off=pop.conn_off)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def tensor(a, device="cuda"):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device)


def bucket_members(pop, tr, buckets):
    """Genome indices of each plan bucket, by the plan's documented rule:
    register buckets by prog_rows (flagged genomes in the first), LDS buckets by
    n_rows for the programs too large for the largest register file."""
    st = host(tr.status)[:pop.P]
    pr = host(tr.prog_rows)[:pop.P]
    nr = host(tr.n_rows)[:pop.P]
    reg = [b["rows_class"] for b in buckets if b["engine"] == 2]
    reg_max = max(reg) if reg else 0
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
