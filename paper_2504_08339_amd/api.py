"""Python face of libtnhip: torch tensors in, device pointers out.

Each function allocates its outputs as torch tensors on the population's device,
passes raw pointers and torch's current HIP stream to the C ABI, and raises
TNError on a non-zero status. No arithmetic of the method happens here.
"""
from __future__ import annotations

import ctypes
import dataclasses
from typing import Optional, Tuple

import numpy as np
import torch

from . import _abi
from ._abi import TNError, TnPopulation, TnTransformed, TnTransformedElems

_lib = _abi.load()

_NODE = {"node_key": torch.int32, "node_bias": torch.float32, "node_resp": torch.float32,
         "node_act": torch.uint8, "node_agg": torch.uint8}
_CONN = {"conn_in": torch.int32, "conn_out": torch.int32, "conn_w": torch.float32,
         "conn_en": torch.uint8}


def lib():
    return _lib


def _p(t, ctype):
    return None if t is None else ctypes.cast(ctypes.c_void_p(t.data_ptr()), ctype)


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _need(t, name, dtype, shape, device):
    """Raises before any launch unless ``t`` is a contiguous ``dtype`` tensor of
    exactly ``shape`` on ``device`` (a host tensor or a short buffer would hand
    a kernel an address it must not read)."""
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if t.device != torch.device(device):
        raise ValueError(f"{name} must be on {device}, got {t.device}")
    if not t.is_contiguous():
        raise TypeError(f"{name} must be contiguous")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return t


def _check(name, rc):
    if rc != _abi.TN_OK:
        text = _lib.tn_status_string(rc).decode()
        if rc == _abi.TN_EHIP:
            text += f" [{_lib.tn_last_error().decode()}]"
        raise TNError(name, rc, text)


class Population:
    """A device-resident population in the library's structure-of-arrays layout.

    Padded: every node tensor is [P][N_max], every connection tensor [P][C_max].
    Ragged: flat tensors plus int64 ``node_off`` / ``conn_off`` of length P+1.
    """

    def __init__(self, n_in: int, n_out: int, N_max: int, C_max: int, tensors: dict,
                 node_off: Optional[torch.Tensor] = None,
                 conn_off: Optional[torch.Tensor] = None):
        self.n_in, self.n_out, self.N_max, self.C_max = int(n_in), int(n_out), int(N_max), int(C_max)
        self.t = {}
        key = tensors["node_key"]
        if not isinstance(key, torch.Tensor) or key.device.type != "cuda":
            raise ValueError("population tensors must be on a GPU device")
        self.device = key.device
        self.node_off, self.conn_off = node_off, conn_off
        if node_off is not None:
            if conn_off is None:
                raise TypeError("node_off and conn_off go together")
            P = node_off.numel() - 1
            for name, o in (("node_off", node_off), ("conn_off", conn_off)):
                _need(o, name, torch.int64, (P + 1,), self.device)
            if P < 0:
                raise ValueError("node_off must hold P+1 >= 1 offsets")
            # the array lengths must be what the offsets say (one read back)
            total_nodes, total_conns = int(node_off[-1]), int(conn_off[-1])
            node_shape, conn_shape = (total_nodes,), (total_conns,)
            self.P = P
        else:
            self.P = key.shape[0] if key.dim() == 2 else 0
            node_shape, conn_shape = (self.P, self.N_max), (self.P, self.C_max)
            total_nodes, total_conns = self.P * self.N_max, self.P * self.C_max
        for name, dt in _NODE.items():
            self.t[name] = _need(tensors[name], name, dt, node_shape, self.device)
        for name, dt in _CONN.items():
            self.t[name] = _need(tensors[name], name, dt, conn_shape, self.device)
        self.c = TnPopulation(
            self.P, self.n_in, self.n_out, self.N_max, self.C_max, total_nodes, total_conns,
            _p(node_off, _abi.c_int64_p), _p(conn_off, _abi.c_int64_p),
            _p(self.t["node_key"], _abi.c_int32_p), _p(self.t["node_bias"], _abi.c_float_p),
            _p(self.t["node_resp"], _abi.c_float_p), _p(self.t["node_act"], _abi.c_uint8_p),
            _p(self.t["node_agg"], _abi.c_uint8_p), _p(self.t["conn_in"], _abi.c_int32_p),
            _p(self.t["conn_out"], _abi.c_int32_p), _p(self.t["conn_w"], _abi.c_float_p),
            _p(self.t["conn_en"], _abi.c_uint8_p))
        _check("tn_validate_population", _lib.tn_validate_population(ctypes.byref(self.c)))

    @property
    def ragged(self) -> bool:
        return self.node_off is not None

    @classmethod
    def from_numpy(cls, n_in, n_out, N_max, C_max, arrays: dict, device="cuda",
                   node_off=None, conn_off=None) -> "Population":
        """Copies host arrays (names as in the C header) to ``device``."""
        def dev(a, dt):
            return torch.from_numpy(np.ascontiguousarray(a)).to(device=device, dtype=dt)
        ts = {k: dev(arrays[k], dt) for k, dt in {**_NODE, **_CONN}.items()}
        if node_off is not None:
            node_off = dev(node_off, torch.int64)
            conn_off = dev(conn_off, torch.int64)
        return cls(n_in, n_out, N_max, C_max, ts, node_off, conn_off)


def pack_paper_layout(PN: torch.Tensor, PC: torch.Tensor, n_in: int, n_out: int,
                      return_errors: bool = False):
    """Population from the paper's float tensors (Section 3.1): PN [P][N_max][5]
    rows [k, bias, response, act, agg], PC [P][C_max][4] rows [k_in, k_out, e, w],
    NaN padding rows anywhere. Raises TNError (TN_EINVAL) when a row breaks the
    encoding's rules, unless ``return_errors``: then returns (population,
    per-genome tn_pack_error bits [P], status code). Synchronises the stream."""
    if not isinstance(PN, torch.Tensor) or PN.dim() != 3 or PN.device.type != "cuda":
        raise ValueError("PN must be a [P][N_max][5] GPU tensor")
    P, N_max, d = PN.shape[0], PN.shape[1], PN.device
    _need(PN, "PN", torch.float32, (P, N_max, 5), d)
    if not isinstance(PC, torch.Tensor) or PC.dim() != 3:
        raise ValueError("PC must be a [P][C_max][4] tensor")
    C_max = PC.shape[1]
    _need(PC, "PC", torch.float32, (P, C_max, 4), d)
    ts = {k: torch.empty((P, N_max), dtype=dt, device=d) for k, dt in _NODE.items()}
    ts.update({k: torch.empty((P, C_max), dtype=dt, device=d) for k, dt in _CONN.items()})
    arrays = _abi.TnPopulationArrays(*[_p(ts[k], ty) for k, ty in (
        ("node_key", _abi.c_int32_p), ("node_bias", _abi.c_float_p),
        ("node_resp", _abi.c_float_p), ("node_act", _abi.c_uint8_p),
        ("node_agg", _abi.c_uint8_p), ("conn_in", _abi.c_int32_p), ("conn_out", _abi.c_int32_p),
        ("conn_w", _abi.c_float_p), ("conn_en", _abi.c_uint8_p))])
    err = torch.empty(max(P, 1), dtype=torch.int32, device=d)
    rc = _lib.tn_pack_paper_layout(_p(PN, _abi.c_float_p), _p(PC, _abi.c_float_p), P, N_max,
                                   C_max, ctypes.byref(arrays), _p(err, _abi.c_int32_p),
                                   _stream(d))
    if not (return_errors and rc == _abi.TN_EINVAL):
        _check("tn_pack_paper_layout", rc)
    pop = Population(n_in, n_out, N_max, C_max, ts)
    return (pop, err[:P], rc) if return_errors else pop


class Transformed:
    """Device tensors written by tn_transform (layout in the C header)."""

    def __init__(self, pop: Population):
        sz = TnTransformedElems()
        _check("tn_transformed_size", _lib.tn_transformed_size(ctypes.byref(pop.c), ctypes.byref(sz)))
        d = pop.device
        i32 = dict(dtype=torch.int32, device=d)
        f32 = dict(dtype=torch.float32, device=d)
        self.status = torch.empty(max(sz.genome_elems, 1), **i32)
        self.n_valid = torch.empty(max(sz.genome_elems, 1), **i32)
        self.order = torch.empty(max(sz.node_elems, 1), **i32)
        self.level = torch.empty(max(sz.node_elems, 1), **i32)
        self.row_ptr = torch.empty(max(sz.rowptr_elems, 1), **i32)
        self.edge_src = torch.empty(max(sz.conn_elems, 1), **i32)
        self.edge_row = torch.empty(max(sz.conn_elems, 1), **i32)
        self.edge_w = torch.empty(max(sz.conn_elems, 1), **f32)
        self.pos_bias = torch.empty(max(sz.node_elems, 1), **f32)
        self.pos_resp = torch.empty(max(sz.node_elems, 1), **f32)
        self.pos_fn = torch.empty(max(sz.node_elems, 1), **i32)
        self.io_pos = torch.empty(max(sz.io_elems, 1), **i32)
        self.pos_row = torch.empty(max(sz.node_elems, 1), **i32)
        self.n_rows = torch.empty(max(sz.genome_elems, 1), **i32)
        self.prog_node = torch.empty(4 * max(sz.node_elems, 1), **i32)
        self.prog_edge = torch.empty(2 * (max(sz.conn_elems, 1) + 8), **i32)  # + 8 padding
        self.prog_edge[-16:].zero_()  # the library never writes the padding: keep it defined
        self.prog_rows = torch.empty(max(sz.genome_elems, 1), **i32)
        self.prog_rec = torch.empty(16 * max(sz.node_elems, 1), **i32)
        self.c = TnTransformed(*[_p(getattr(self, n), ty) for n, ty in (
            ("status", _abi.c_int32_p), ("n_valid", _abi.c_int32_p), ("order", _abi.c_int32_p),
            ("level", _abi.c_int32_p), ("row_ptr", _abi.c_int32_p), ("edge_src", _abi.c_int32_p),
            ("edge_row", _abi.c_int32_p), ("edge_w", _abi.c_float_p), ("pos_bias", _abi.c_float_p),
            ("pos_resp", _abi.c_float_p), ("pos_fn", _abi.c_int32_p), ("io_pos", _abi.c_int32_p),
            ("pos_row", _abi.c_int32_p), ("n_rows", _abi.c_int32_p),
            ("prog_node", _abi.c_int32_p), ("prog_edge", _abi.c_int32_p),
            ("prog_rows", _abi.c_int32_p), ("prog_rec", _abi.c_int32_p))])


def transform(pop: Population, out: Optional[Transformed] = None) -> Transformed:
    tr = out if out is not None else Transformed(pop)
    _check("tn_transform", _lib.tn_transform(ctypes.byref(pop.c), ctypes.byref(tr.c),
                                             _stream(pop.device)))
    return tr


def _obs_stride(pop: Population, obs: torch.Tensor):
    """(B, per-genome stride) of observations [B][n_in] (shared) or [P][B][n_in]."""
    if not isinstance(obs, torch.Tensor) or obs.dim() not in (2, 3):
        raise ValueError("obs must be [B][n_in] (shared) or [P][B][n_in]")
    B = obs.shape[-2]
    if obs.dim() == 2:
        _need(obs, "obs", torch.float32, (B, pop.n_in), pop.device)
        return B, 0
    _need(obs, "obs", torch.float32, (pop.P, B, pop.n_in), pop.device)
    return B, B * pop.n_in


def _per_genome(pop: Population, t: torch.Tensor, name: str, B: int):
    """Stride of a [B][n_out] (shared) or [P][B][n_out] float32 tensor."""
    if not isinstance(t, torch.Tensor) or t.dim() not in (2, 3):
        raise ValueError(f"{name} must be [B][n_out] (shared) or [P][B][n_out]")
    if t.dim() == 2:
        _need(t, name, torch.float32, (B, pop.n_out), pop.device)
        return 0
    _need(t, name, torch.float32, (pop.P, B, pop.n_out), pop.device)
    return B * pop.n_out


def _out(pop: Population, out, B: int):
    shape = (pop.P, B, pop.n_out)
    if out is None:
        return torch.empty(shape, dtype=torch.float32, device=pop.device)
    return _need(out, "out", torch.float32, shape, pop.device)


def forward(pop: Population, tr: Transformed, obs: torch.Tensor,
            out: Optional[torch.Tensor] = None, engine: int = 0, obs_per_lane: int = 0,
            waves_per_genome: int = 0, rows: int = 0) -> torch.Tensor:
    """Outputs [P][B][n_out] of every genome on obs ([B][n_in] shared or [P][B][n_in]).
    ``engine`` (TN_ENGINE_AUTO / LDS / REG), ``obs_per_lane``, ``waves_per_genome``
    and ``rows`` only change how the work is laid out on the chip (0 = library
    choice); a genome needing more value rows than ``rows`` gets NaN outputs."""
    B, stride = _obs_stride(pop, obs)
    out = _out(pop, out, B)
    tile = _abi.TnTile(engine, obs_per_lane, waves_per_genome, rows)
    _check("tn_forward_tiled", _lib.tn_forward_tiled(
        ctypes.byref(pop.c), ctypes.byref(tr.c), _p(obs, _abi.c_float_p), stride, B,
        _p(out, _abi.c_float_p), ctypes.byref(tile), _stream(pop.device)))
    return out


def forward_recurrent(pop: Population, obs: torch.Tensor, T: int,
                      out: Optional[torch.Tensor] = None, with_status: bool = False):
    """Outputs [P][B][n_out] of recurrent networks after T synchronous sweeps
    (tn_forward_recurrent; no transformation needed). With ``with_status`` also
    the per-genome status bits [P] (cycles allowed)."""
    B, stride = _obs_stride(pop, obs)
    out = _out(pop, out, B)
    status = torch.empty(max(pop.P, 1), dtype=torch.int32, device=pop.device) if with_status else None
    _check("tn_forward_recurrent", _lib.tn_forward_recurrent(
        ctypes.byref(pop.c), _p(obs, _abi.c_float_p), stride, B, int(T), _p(out, _abi.c_float_p),
        _p(status, _abi.c_int32_p), _stream(pop.device)))
    return (out, status[:pop.P]) if with_status else out


def forward_loss(pop: Population, tr: Transformed, obs: torch.Tensor, target: torch.Tensor,
                 scale: float = 1.0, offset: float = 0.0, store_outputs: bool = True):
    """(loss [P], outputs or None): loss[g] = offset + scale * sum (y - target)^2."""
    B, stride = _obs_stride(pop, obs)
    tstride = _per_genome(pop, target, "target", B)
    out = (torch.empty((pop.P, B, pop.n_out), dtype=torch.float32, device=pop.device)
           if store_outputs else None)
    loss = torch.empty(max(pop.P, 1), dtype=torch.float32, device=pop.device)
    _check("tn_forward_loss", _lib.tn_forward_loss(
        ctypes.byref(pop.c), ctypes.byref(tr.c), _p(obs, _abi.c_float_p), stride, B,
        _p(target, _abi.c_float_p), tstride, scale, offset, _p(out, _abi.c_float_p),
        _p(loss, _abi.c_float_p), _stream(pop.device)))
    return loss[:pop.P], out


def _grad_buffers(pop: Population):
    dW = torch.empty_like(pop.t["conn_w"])
    db = torch.empty_like(pop.t["node_bias"])
    return dW, db


def backward(pop: Population, tr: Transformed, obs: torch.Tensor, dY: torch.Tensor):
    """(dW, db) shaped like conn_w / node_bias, for upstream gradient dY [P][B][n_out]."""
    B, stride = _obs_stride(pop, obs)
    _need(dY, "dY", torch.float32, (pop.P, B, pop.n_out), pop.device)
    dW, db = _grad_buffers(pop)
    _check("tn_backward", _lib.tn_backward(
        ctypes.byref(pop.c), ctypes.byref(tr.c), _p(obs, _abi.c_float_p), stride, B,
        _p(dY, _abi.c_float_p), B * pop.n_out, _p(dW, _abi.c_float_p), _p(db, _abi.c_float_p),
        _stream(pop.device)))
    return dW, db


def forward_backward_mse(pop: Population, tr: Transformed, obs: torch.Tensor,
                         target: torch.Tensor):
    """(loss [P], dW, db): mean squared error against target ([B][n_out] shared or
    [P][B][n_out]) and its gradient with respect to weights and biases."""
    B, stride = _obs_stride(pop, obs)
    tstride = _per_genome(pop, target, "target", B)
    dW, db = _grad_buffers(pop)
    loss = torch.empty(max(pop.P, 1), dtype=torch.float32, device=pop.device)
    _check("tn_forward_backward_mse", _lib.tn_forward_backward_mse(
        ctypes.byref(pop.c), ctypes.byref(tr.c), _p(obs, _abi.c_float_p), stride, B,
        _p(target, _abi.c_float_p), tstride, _p(loss, _abi.c_float_p), _p(dW, _abi.c_float_p),
        _p(db, _abi.c_float_p), _stream(pop.device)))
    return loss[:pop.P], dW, db


class DistanceWorkspace:
    def __init__(self, pop: Population):
        n = ctypes.c_size_t()
        _check("tn_distance_workspace_size",
               _lib.tn_distance_workspace_size(ctypes.byref(pop.c), ctypes.byref(n)))
        self.nbytes = int(n.value)
        self.buf = torch.empty(max(self.nbytes, 1), dtype=torch.uint8, device=pop.device)


def _distance_outputs(pop: Population, counts: bool, out):
    P = pop.P
    if out is None:
        dist = torch.empty((P, P), dtype=torch.float32, device=pop.device)
        E = torch.empty((P, P), dtype=torch.int32, device=pop.device) if counts else None
        D = torch.empty((P, P), dtype=torch.int32, device=pop.device) if counts else None
    else:
        dist, E, D = out
        _need(dist, "dist", torch.float32, (P, P), pop.device)
        if (E is None) != (D is None):
            raise ValueError("excess and disjoint go together")
        if E is not None:
            _need(E, "excess", torch.int32, (P, P), pop.device)
            _need(D, "disjoint", torch.int32, (P, P), pop.device)
    return dist, E, D


def distance(pop: Population, c1: float = 1.0, c2: float = 1.0, c3: float = 0.4,
             counts: bool = True, workspace: Optional[DistanceWorkspace] = None, out=None):
    """(dist [P][P], excess [P][P] or None, disjoint [P][P] or None)."""
    ws = workspace if workspace is not None else DistanceWorkspace(pop)
    dist, E, D = _distance_outputs(pop, counts, out)
    if ws.buf.device != pop.device or ws.buf.numel() < ws.nbytes:
        raise ValueError("distance workspace from another population or device")
    _check("tn_distance", _lib.tn_distance(
        ctypes.byref(pop.c), c1, c2, c3, ctypes.c_void_p(ws.buf.data_ptr()),
        _p(dist, _abi.c_float_p), _p(E, _abi.c_int32_p), _p(D, _abi.c_int32_p),
        _stream(pop.device)))
    return dist, E, D


def distance_noalloc(pop: Population, c1: float = 1.0, c2: float = 1.0, c3: float = 0.4,
                     counts: bool = True, out=None):
    """distance() through tn_distance_noalloc: the library's fixed device scratch
    instead of a workspace (no device allocation by the call; pass ``out`` to
    allocate nothing here either)."""
    dist, E, D = _distance_outputs(pop, counts, out)
    _check("tn_distance_noalloc", _lib.tn_distance_noalloc(
        ctypes.byref(pop.c), c1, c2, c3, _p(dist, _abi.c_float_p), _p(E, _abi.c_int32_p),
        _p(D, _abi.c_int32_p), _stream(pop.device)))
    return dist, E, D


def distance_nodes(pop: Population, c_disjoint: float = 1.0, c_homologous: float = 0.5,
                   counts: bool = True, out=None):
    """(dist [P][P], D_nodes [P][P] or None, D_conns [P][P] or None): the
    node-inclusive distance of tn_distance_nodes."""
    n = ctypes.c_size_t()
    _check("tn_distance_nodes_workspace_size",
           _lib.tn_distance_nodes_workspace_size(ctypes.byref(pop.c), ctypes.byref(n)))
    ws = torch.empty(max(int(n.value), 1), dtype=torch.uint8, device=pop.device)
    dist, DN, DC = _distance_outputs(pop, counts, out)
    _check("tn_distance_nodes", _lib.tn_distance_nodes(
        ctypes.byref(pop.c), c_disjoint, c_homologous, ctypes.c_void_p(ws.data_ptr()),
        _p(dist, _abi.c_float_p), _p(DN, _abi.c_int32_p), _p(DC, _abi.c_int32_p),
        _stream(pop.device)))
    return dist, DN, DC


@dataclasses.dataclass
class MutationParams:
    """Reproduction hyperparameters (Appendix A; defaults of Appendix C's
    feedforward setting: tanh hidden nodes, sum aggregation)."""
    node_add: float = 0.2
    node_delete: float = 0.0
    conn_add: float = 0.4
    conn_delete: float = 0.0
    bias_init_mean: float = 0.0
    bias_init_std: float = 1.0
    bias_mutate_power: float = 0.5
    bias_mutate_rate: float = 0.7
    bias_replace_rate: float = 0.1
    resp_init_mean: float = 1.0
    resp_init_std: float = 0.0
    resp_mutate_power: float = 0.0
    resp_mutate_rate: float = 0.0
    resp_replace_rate: float = 0.0
    weight_init_mean: float = 0.0
    weight_init_std: float = 1.0
    weight_mutate_power: float = 0.5
    weight_mutate_rate: float = 0.8
    weight_replace_rate: float = 0.1
    act_default: int = 2
    agg_default: int = 0
    act_replace_rate: float = 0.0
    agg_replace_rate: float = 0.0
    act_options: Tuple[int, ...] = (2,)
    agg_options: Tuple[int, ...] = (0,)
    allow_cycles: bool = False

    def to_c(self) -> "_abi.TnMutationParams":
        c = _abi.TnMutationParams()
        for f in dataclasses.fields(self):
            if f.name in ("act_options", "agg_options"):
                opts = sorted(int(o) for o in getattr(self, f.name))
                if not 1 <= len(opts) <= 8:
                    raise ValueError(f"{f.name}: 1 to 8 codes")
                arr = getattr(c, f.name)
                for i, o in enumerate(opts):
                    arr[i] = o
                setattr(c, "n_" + f.name, len(opts))
            elif f.name == "allow_cycles":
                c.allow_cycles = int(bool(self.allow_cycles))
            else:
                setattr(c, f.name, getattr(self, f.name))
        return c


def _padded_arrays(n: int, N_max: int, C_max: int, device):
    """Fresh [n][N_max] / [n][C_max] tensors and their tn_population_arrays."""
    ts = {k: torch.empty((n, N_max), dtype=dt, device=device) for k, dt in _NODE.items()}
    ts.update({k: torch.empty((n, C_max), dtype=dt, device=device) for k, dt in _CONN.items()})
    arrays = _abi.TnPopulationArrays(*[_p(ts[k], ty) for k, ty in (
        ("node_key", _abi.c_int32_p), ("node_bias", _abi.c_float_p),
        ("node_resp", _abi.c_float_p), ("node_act", _abi.c_uint8_p),
        ("node_agg", _abi.c_uint8_p), ("conn_in", _abi.c_int32_p), ("conn_out", _abi.c_int32_p),
        ("conn_w", _abi.c_float_p), ("conn_en", _abi.c_uint8_p))])
    return ts, arrays


def reproduce_draws(N_max: int, C_max: int):
    """(uniforms, normals) tn_reproduce reads per child."""
    nu, nz = ctypes.c_int32(), ctypes.c_int32()
    _check("tn_reproduce_draws", _lib.tn_reproduce_draws(N_max, C_max, ctypes.byref(nu),
                                                          ctypes.byref(nz)))
    return int(nu.value), int(nz.value)


def reproduce(pop: Population, parents: torch.Tensor, U: torch.Tensor, Z: torch.Tensor,
              params: Optional[MutationParams] = None, next_key: int = 0):
    """Children of a padded population by crossover and mutation (tn_reproduce):
    parents int32 [n][2] (fitter first; a second parent of -1 copies the first),
    draws U [n][n_uniform], Z [n][n_normal] float32. Returns (children as a
    Population with the parents' capacities, next unused key as a device int32
    tensor [1])."""
    if pop.ragged:
        raise ValueError("reproduce takes a padded population")
    d = pop.device
    if not isinstance(parents, torch.Tensor) or parents.dim() != 2:
        raise ValueError("parents must be an int32 [n][2] tensor")
    n = parents.shape[0]
    nu, nz = reproduce_draws(pop.N_max, pop.C_max)
    _need(parents, "parents", torch.int32, (n, 2), d)
    _need(U, "U", torch.float32, (n, nu), d)
    _need(Z, "Z", torch.float32, (n, nz), d)
    prm = (params or MutationParams()).to_c()
    ts, arrays = _padded_arrays(n, pop.N_max, pop.C_max, d)
    nb = ctypes.c_size_t()
    _check("tn_reproduce_workspace_size", _lib.tn_reproduce_workspace_size(n, ctypes.byref(nb)))
    ws = torch.empty(max(int(nb.value), 1), dtype=torch.uint8, device=d)
    nk = torch.empty(1, dtype=torch.int32, device=d)
    _check("tn_reproduce", _lib.tn_reproduce(
        ctypes.byref(pop.c), n, _p(parents, _abi.c_int32_p), _p(U, _abi.c_float_p),
        _p(Z, _abi.c_float_p), ctypes.byref(prm), int(next_key), ctypes.byref(arrays),
        _p(nk, _abi.c_int32_p), ctypes.c_void_p(ws.data_ptr()), _stream(d)))
    return Population(pop.n_in, pop.n_out, pop.N_max, pop.C_max, ts), nk


@dataclasses.dataclass
class NeatParams:
    """Generation hyperparameters (Appendix A; values of Appendix C)."""
    compatibility_threshold: float = 3.5
    compatibility_disjoint: float = 1.0
    compatibility_homologous: float = 0.5
    max_species: int = 10
    species_elitism: int = 2
    max_stagnation: int = 15
    genome_elitism: int = 2
    survival_threshold: float = 0.2
    spawn_number_change_rate: float = 0.5
    mutation: MutationParams = dataclasses.field(default_factory=MutationParams)

    def to_c(self) -> "_abi.TnNeatParams":
        c = _abi.TnNeatParams()
        for f in dataclasses.fields(self):
            if f.name == "mutation":
                c.mutation = self.mutation.to_c()
            else:
                setattr(c, f.name, getattr(self, f.name))
        return c


class SpeciesTable:
    """Device species table (tn_species_table): representatives [S][N_max] /
    [S][C_max] and per-slot alive, best, last_improved, size."""

    def __init__(self, max_species: int, N_max: int, C_max: int, device):
        self.max_species = int(max_species)
        self.reps, arrays = _padded_arrays(self.max_species, N_max, C_max, device)
        i32 = dict(dtype=torch.int32, device=device)
        self.alive = torch.zeros(self.max_species, **i32)
        self.best = torch.full((self.max_species,), float("-inf"), dtype=torch.float32,
                               device=device)
        self.last_improved = torch.zeros(self.max_species, **i32)
        self.size = torch.zeros(self.max_species, **i32)
        self.c = _abi.TnSpeciesTable(self.max_species, arrays, _p(self.alive, _abi.c_int32_p),
                                     _p(self.best, _abi.c_float_p),
                                     _p(self.last_improved, _abi.c_int32_p),
                                     _p(self.size, _abi.c_int32_p))


def neat_init(P: int, n_in: int, n_out: int, N_max: int, C_max: int, Z: torch.Tensor,
              mutation: Optional[MutationParams] = None, max_species: Optional[int] = None):
    """(initial population, cleared species table) of tn_neat_init; Z [P][n_normal]."""
    d = Z.device
    _, nz = reproduce_draws(N_max, C_max)
    _need(Z, "Z", torch.float32, (P, nz), d)
    m = mutation or MutationParams()
    ts, arrays = _padded_arrays(P, N_max, C_max, d)
    table = SpeciesTable(max_species or NeatParams().max_species, N_max, C_max, d)
    _check("tn_neat_init", _lib.tn_neat_init(P, n_in, n_out, N_max, C_max, _p(Z, _abi.c_float_p),
                                             ctypes.byref(m.to_c()), ctypes.byref(arrays),
                                             ctypes.byref(table.c), _stream(d)))
    return Population(n_in, n_out, N_max, C_max, ts), table


def neat_generation(pop: Population, fitness: torch.Tensor, generation: int,
                    table: SpeciesTable, sel: torch.Tensor, U: torch.Tensor, Z: torch.Tensor,
                    next_key, params: Optional[NeatParams] = None):
    """One generation (tn_neat_generation): returns (children, species_of [P],
    parents [P][2], next unused key as a device int32 tensor [1]). ``next_key``
    is an int. The table is updated in place."""
    prm = params or NeatParams()
    if table.max_species != prm.max_species:
        raise ValueError("table and params disagree on max_species")
    if pop.ragged:
        raise ValueError("neat_generation takes a padded population")
    d, P = pop.device, pop.P
    nu, nz = reproduce_draws(pop.N_max, pop.C_max)
    _need(fitness, "fitness", torch.float32, (P,), d)
    _need(sel, "sel", torch.float32, (P, 2), d)
    _need(U, "U", torch.float32, (P, nu), d)
    _need(Z, "Z", torch.float32, (P, nz), d)
    if table.reps["node_key"].shape != (table.max_species, pop.N_max) or \
            table.reps["conn_in"].shape != (table.max_species, pop.C_max) or \
            table.alive.device != torch.device(d):
        raise ValueError("species table shaped for another population or device")
    ts, arrays = _padded_arrays(P, pop.N_max, pop.C_max, d)
    nb = ctypes.c_size_t()
    _check("tn_neat_workspace_size", _lib.tn_neat_workspace_size(
        ctypes.byref(pop.c), prm.max_species, ctypes.byref(nb)))
    ws = torch.empty(max(int(nb.value), 1), dtype=torch.uint8, device=d)
    sp = torch.empty(P, dtype=torch.int32, device=d)
    par = torch.empty((P, 2), dtype=torch.int32, device=d)
    nk = torch.empty(1, dtype=torch.int32, device=d)
    _check("tn_neat_generation", _lib.tn_neat_generation(
        ctypes.byref(pop.c), _p(fitness, _abi.c_float_p), int(generation),
        ctypes.byref(prm.to_c()), ctypes.byref(table.c), _p(sel, _abi.c_float_p),
        _p(U, _abi.c_float_p), _p(Z, _abi.c_float_p), int(next_key), ctypes.byref(arrays),
        _p(sp, _abi.c_int32_p), _p(par, _abi.c_int32_p), _p(nk, _abi.c_int32_p),
        ctypes.c_void_p(ws.data_ptr()), _stream(d)))
    return Population(pop.n_in, pop.n_out, pop.N_max, pop.C_max, ts), sp, par, nk


class Plan:
    """Batched forward pass over length buckets (tn_plan_*): ``forward`` replays
    the persistent per-bucket kernels captured in a hipGraph, ``forward_buckets``
    launches one plain kernel per bucket; both give tn_forward's bits. The
    population and transformed tensors must stay alive and unchanged."""

    def __init__(self, pop: Population, tr: Transformed, B: int,
                 tune_cache: Optional[str] = None):
        self.pop, self.tr, self.B = pop, tr, int(B)
        self._h = ctypes.c_void_p()
        _check("tn_plan_create", _lib.tn_plan_create(
            ctypes.byref(pop.c), ctypes.byref(tr.c), self.B,
            tune_cache.encode() if tune_cache else None, ctypes.byref(self._h),
            _stream(pop.device)))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.tn_plan_destroy(h)
            self._h = ctypes.c_void_p()

    def buckets(self):
        out = []
        for i in range(_lib.tn_plan_num_buckets(self._h)):
            info = _abi.TnBucketInfo()
            _check("tn_plan_bucket", _lib.tn_plan_bucket(self._h, i, ctypes.byref(info)))
            out.append({"engine": info.engine, "rows_class": info.rows_class,
                        "count": info.count, "edges": int(info.edges),
                        "obs_per_lane": info.tile.obs_per_lane,
                        "waves": info.tile.waves_per_genome, "rows": info.tile.rows})
        return out

    def set_tile(self, i: int, obs_per_lane: int, waves: int):
        _check("tn_plan_set_tile", _lib.tn_plan_set_tile(self._h, i, obs_per_lane, waves))

    def _call(self, name, obs, out):
        B, stride = _obs_stride(self.pop, obs)
        if B != self.B:
            raise ValueError(f"the plan was made for B={self.B}, got {B}")
        out = _out(self.pop, out, B)
        _check(name, getattr(_lib, name)(self._h, _p(obs, _abi.c_float_p), stride,
                                         _p(out, _abi.c_float_p), _stream(self.pop.device)))
        return out

    def forward(self, obs: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        return self._call("tn_plan_forward", obs, out)

    def forward_buckets(self, obs: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        return self._call("tn_plan_forward_buckets", obs, out)

    def forward_bucket(self, i: int, obs: torch.Tensor, out: torch.Tensor,
                       persistent: bool = True) -> torch.Tensor:
        B, stride = _obs_stride(self.pop, obs)
        if B != self.B:
            raise ValueError(f"the plan was made for B={self.B}, got {B}")
        out = _out(self.pop, out, B)
        _check("tn_plan_forward_bucket", _lib.tn_plan_forward_bucket(
            self._h, i, 1 if persistent else 0, _p(obs, _abi.c_float_p), stride,
            _p(out, _abi.c_float_p), _stream(self.pop.device)))
        return out

    def tune(self, obs: torch.Tensor, out: Optional[torch.Tensor] = None,
             tune_cache: Optional[str] = None) -> None:
        B, stride = _obs_stride(self.pop, obs)
        if B != self.B:
            raise ValueError(f"the plan was made for B={self.B}, got {B}")
        out = _out(self.pop, out, B)
        _check("tn_plan_tune", _lib.tn_plan_tune(
            self._h, _p(obs, _abi.c_float_p), stride, _p(out, _abi.c_float_p),
            tune_cache.encode() if tune_cache else None, _stream(self.pop.device)))


def _substrate(grid: int, n_out: int, threshold: float):
    return _abi.TnSubstrate(int(grid), int(n_out), float(threshold))


def cppn_query(pop: Population, tr: Transformed, grid: int = 32, n_out: int = 8,
               threshold: float = 0.2, raw: bool = False):
    """(w1t [P][S][S], w2t [P][n_out][S]) bfloat16 substrate weights of every
    CPPN genome (transposed: row = target), plus (raw1, raw2) float32 CPPN values
    before the threshold when ``raw``."""
    sub = _substrate(grid, n_out, threshold)
    S = int(grid) * int(grid)
    P, d = pop.P, pop.device
    w1t = torch.empty((P, S, S), dtype=torch.bfloat16, device=d)
    w2t = torch.empty((P, n_out, S), dtype=torch.bfloat16, device=d)
    r1 = torch.empty((P, S, S), dtype=torch.float32, device=d) if raw else None
    r2 = torch.empty((P, n_out, S), dtype=torch.float32, device=d) if raw else None
    _check("tn_cppn_query", _lib.tn_cppn_query(
        ctypes.byref(pop.c), ctypes.byref(tr.c), ctypes.byref(sub),
        ctypes.c_void_p(w1t.data_ptr()), ctypes.c_void_p(w2t.data_ptr()),
        _p(r1, _abi.c_float_p), _p(r2, _abi.c_float_p), _stream(d)))
    return (w1t, w2t, r1, r2) if raw else (w1t, w2t)


def _x_layout(x: torch.Tensor, P: int, S: int):
    """(B, stride) of substrate inputs x: [B][S] shared or [P][B][S] bfloat16."""
    if not isinstance(x, torch.Tensor) or x.dim() not in (2, 3):
        raise ValueError("x must be [B][S] (shared) or [P][B][S]")
    B = x.shape[-2]
    if x.dim() == 2:
        _need(x, "x", torch.bfloat16, (B, S), x.device)
        return B, 0
    _need(x, "x", torch.bfloat16, (P, B, S), x.device)
    return B, B * S


def substrate_forward(w1t: torch.Tensor, w2t: torch.Tensor, x: torch.Tensor, grid: int = 32,
                      n_out: int = 8, threshold: float = 0.2):
    """(h [P][B][S] float32, y [P][B][n_out] float32) for bfloat16 inputs x
    ([B][S] shared or [P][B][S])."""
    sub = _substrate(grid, n_out, threshold)
    S = int(grid) * int(grid)
    if not isinstance(w1t, torch.Tensor) or w1t.dim() != 3 or w1t.device.type != "cuda":
        raise ValueError("w1t must be a [P][S][S] GPU tensor")
    P, d = w1t.shape[0], w1t.device
    _need(w1t, "w1t", torch.bfloat16, (P, S, S), d)
    _need(w2t, "w2t", torch.bfloat16, (P, n_out, S), d)
    B, stride = _x_layout(x, P, S)
    if x.device != d:
        raise ValueError("x must be on the weights' device")
    h = torch.empty((P, B, S), dtype=torch.float32, device=d)
    y = torch.empty((P, B, n_out), dtype=torch.float32, device=d)
    _check("tn_substrate_forward", _lib.tn_substrate_forward(
        ctypes.byref(sub), P, ctypes.c_void_p(w1t.data_ptr()), ctypes.c_void_p(w2t.data_ptr()),
        ctypes.c_void_p(x.data_ptr()), stride, B, _p(h, _abi.c_float_p), _p(y, _abi.c_float_p),
        _stream(d)))
    return h, y


def substrate_backward(w2t: torch.Tensor, x: torch.Tensor, h: torch.Tensor, dy: torch.Tensor,
                       grid: int = 32, n_out: int = 8, threshold: float = 0.2):
    """(dw1t [P][S][S], dw2t [P][n_out][S]) float32: gradient of sum(dy * y)
    with respect to the substrate weights the forward used."""
    sub = _substrate(grid, n_out, threshold)
    S = int(grid) * int(grid)
    if not isinstance(w2t, torch.Tensor) or w2t.dim() != 3 or w2t.device.type != "cuda":
        raise ValueError("w2t must be a [P][n_out][S] GPU tensor")
    P, d = w2t.shape[0], w2t.device
    _need(w2t, "w2t", torch.bfloat16, (P, n_out, S), d)
    B, stride = _x_layout(x, P, S)
    if x.device != d:
        raise ValueError("x must be on the weights' device")
    _need(h, "h", torch.float32, (P, B, S), d)
    _need(dy, "dy", torch.float32, (P, B, n_out), d)
    n = ctypes.c_size_t()
    _check("tn_substrate_workspace_size", _lib.tn_substrate_workspace_size(
        ctypes.byref(sub), P, B, stride, ctypes.byref(n)))
    ws = torch.empty(max(int(n.value), 1), dtype=torch.uint8, device=d)
    dw1t = torch.empty((P, S, S), dtype=torch.float32, device=d)
    dw2t = torch.empty((P, n_out, S), dtype=torch.float32, device=d)
    _check("tn_substrate_backward", _lib.tn_substrate_backward(
        ctypes.byref(sub), P, ctypes.c_void_p(w2t.data_ptr()), ctypes.c_void_p(x.data_ptr()),
        stride, B, _p(h, _abi.c_float_p), _p(dy, _abi.c_float_p), ctypes.c_void_p(ws.data_ptr()),
        _p(dw1t, _abi.c_float_p), _p(dw2t, _abi.c_float_p), _stream(d)))
    return dw1t, dw2t


def cppn_backward(pop: Population, tr: Transformed, dw1t: torch.Tensor, dw2t: torch.Tensor,
                  grid: int = 32, n_out: int = 8, threshold: float = 0.2):
    """(dW, db) shaped like conn_w / node_bias: gradient of sum(dw * w) over every
    substrate weight the CPPNs produce, through the weights that survived the
    threshold (dw1t [P][S][S], dw2t [P][n_out][S] float32, as from
    substrate_backward)."""
    sub = _substrate(grid, n_out, threshold)
    S = int(grid) * int(grid)
    _need(dw1t, "dw1t", torch.float32, (pop.P, S, S), pop.device)
    _need(dw2t, "dw2t", torch.float32, (pop.P, n_out, S), pop.device)
    n = ctypes.c_size_t()
    _check("tn_cppn_backward_workspace_size", _lib.tn_cppn_backward_workspace_size(
        ctypes.byref(pop.c), ctypes.byref(sub), ctypes.byref(n)))
    ws = torch.empty(max(int(n.value), 1), dtype=torch.uint8, device=pop.device)
    dW, db = _grad_buffers(pop)
    _check("tn_cppn_backward", _lib.tn_cppn_backward(
        ctypes.byref(pop.c), ctypes.byref(tr.c), ctypes.byref(sub), _p(dw1t, _abi.c_float_p),
        _p(dw2t, _abi.c_float_p), ctypes.c_void_p(ws.data_ptr()), _p(dW, _abi.c_float_p),
        _p(db, _abi.c_float_p), _stream(pop.device)))
    return dW, db
