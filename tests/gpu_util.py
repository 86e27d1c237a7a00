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
