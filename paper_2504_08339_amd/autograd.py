"""torch.autograd.Function over the library's forward pass and adjoint.

TNForward.apply(pop, obs, conn_w, node_bias) returns the outputs [P][B][n_out]
of every genome, treating the connection weights and node biases as
differentiable inputs; its backward calls tn_backward. The topology (and every
other attribute) comes from ``pop``; the weights and biases passed in replace
pop's own for this call.
"""
from __future__ import annotations

import torch

from . import api


def _with_params(pop: api.Population, conn_w: torch.Tensor, node_bias: torch.Tensor):
    ts = dict(pop.t)
    ts["conn_w"] = conn_w.detach().contiguous()
    ts["node_bias"] = node_bias.detach().contiguous()
    return api.Population(pop.n_in, pop.n_out, pop.N_max, pop.C_max, ts, pop.node_off, pop.conn_off)


class TNForward(torch.autograd.Function):
    @staticmethod
    def forward(ctx, pop, obs, conn_w, node_bias):
        p = _with_params(pop, conn_w, node_bias)
        tr = api.transform(p)
        y = api.forward(p, tr, obs)
        ctx.saved = (p, tr, obs)
        return y

    @staticmethod
    def backward(ctx, dY):
        p, tr, obs = ctx.saved
        dW, db = api.backward(p, tr, obs, dY.contiguous())
        return None, None, dW, db
