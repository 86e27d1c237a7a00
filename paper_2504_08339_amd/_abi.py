"""ctypes mirror of include/tensorneat_hip.h and the loader of libtnhip.so.

Argument marshalling only: every computation happens in the HIP library. A
missing library is an ImportError (there is no fallback path).
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtnhip.so")

c_int32_p = ctypes.POINTER(ctypes.c_int32)
c_int64_p = ctypes.POINTER(ctypes.c_int64)
c_float_p = ctypes.POINTER(ctypes.c_float)
c_uint8_p = ctypes.POINTER(ctypes.c_uint8)

TN_OK, TN_EINVAL, TN_ESHAPE, TN_EUNSUPPORTED, TN_EHIP, TN_ENOMEM = range(6)
TN_MAX_NODES, TN_MAX_CONNS, TN_MAX_IO = 1024, 4096, 1024

# per-genome status bits
TN_CYCLE, TN_DANGLING, TN_DUP_CONN, TN_DUP_NODE = 1, 2, 4, 8
TN_INPUT_DST, TN_MISSING_IO, TN_OVERSIZE, TN_BAD_ATTR = 16, 32, 64, 128
TN_ENGINE_AUTO, TN_ENGINE_LDS, TN_ENGINE_REG = 0, 1, 2
# tn_pack_paper_layout error bits
TN_PACK_NODE_KEY, TN_PACK_NODE_CODE, TN_PACK_CONN_KEY, TN_PACK_CONN_FLAG = 1, 2, 4, 8


class TnPopulation(ctypes.Structure):
    _fields_ = [
        ("P", ctypes.c_int32), ("n_in", ctypes.c_int32), ("n_out", ctypes.c_int32),
        ("N_max", ctypes.c_int32), ("C_max", ctypes.c_int32),
        ("total_nodes", ctypes.c_int64), ("total_conns", ctypes.c_int64),
        ("node_off", c_int64_p), ("conn_off", c_int64_p),
        ("node_key", c_int32_p), ("node_bias", c_float_p), ("node_resp", c_float_p),
        ("node_act", c_uint8_p), ("node_agg", c_uint8_p),
        ("conn_in", c_int32_p), ("conn_out", c_int32_p), ("conn_w", c_float_p),
        ("conn_en", c_uint8_p),
    ]


class TnTransformed(ctypes.Structure):
    _fields_ = [(n, c_int32_p) for n in ("status", "n_valid", "order", "level", "row_ptr",
                                         "edge_src", "edge_row")] + [
        ("edge_w", c_float_p), ("pos_bias", c_float_p), ("pos_resp", c_float_p),
        ("pos_fn", c_int32_p), ("io_pos", c_int32_p), ("pos_row", c_int32_p),
        ("n_rows", c_int32_p), ("prog_node", c_int32_p), ("prog_edge", c_int32_p),
        ("prog_rows", c_int32_p), ("prog_rec", c_int32_p)]


class TnTransformedElems(ctypes.Structure):
    _fields_ = [("node_elems", ctypes.c_int64), ("rowptr_elems", ctypes.c_int64),
                ("conn_elems", ctypes.c_int64), ("genome_elems", ctypes.c_int64),
                ("io_elems", ctypes.c_int64)]


class TnPopulationArrays(ctypes.Structure):
    _fields_ = [("node_key", c_int32_p), ("node_bias", c_float_p), ("node_resp", c_float_p),
                ("node_act", c_uint8_p), ("node_agg", c_uint8_p), ("conn_in", c_int32_p),
                ("conn_out", c_int32_p), ("conn_w", c_float_p), ("conn_en", c_uint8_p)]


class TnTile(ctypes.Structure):
    _fields_ = [("engine", ctypes.c_int32), ("obs_per_lane", ctypes.c_int32),
                ("waves_per_genome", ctypes.c_int32), ("rows", ctypes.c_int32)]


class TnSubstrate(ctypes.Structure):
    _fields_ = [("grid", ctypes.c_int32), ("n_out", ctypes.c_int32), ("threshold", ctypes.c_float)]


class TnMutationParams(ctypes.Structure):
    _fields_ = ([(n, ctypes.c_float) for n in (
        "node_add", "node_delete", "conn_add", "conn_delete",
        "bias_init_mean", "bias_init_std", "bias_mutate_power", "bias_mutate_rate",
        "bias_replace_rate", "resp_init_mean", "resp_init_std", "resp_mutate_power",
        "resp_mutate_rate", "resp_replace_rate", "weight_init_mean", "weight_init_std",
        "weight_mutate_power", "weight_mutate_rate", "weight_replace_rate",
        "act_replace_rate", "agg_replace_rate")] +
        [(n, ctypes.c_int32) for n in ("act_default", "agg_default", "n_act_options",
                                       "n_agg_options")] +
        [("act_options", ctypes.c_uint8 * 8), ("agg_options", ctypes.c_uint8 * 8),
         ("allow_cycles", ctypes.c_int32)])


class TnNeatParams(ctypes.Structure):
    _fields_ = [("compatibility_threshold", ctypes.c_float), ("compatibility_disjoint", ctypes.c_float),
                ("compatibility_homologous", ctypes.c_float), ("max_species", ctypes.c_int32),
                ("species_elitism", ctypes.c_int32), ("max_stagnation", ctypes.c_int32),
                ("genome_elitism", ctypes.c_int32), ("survival_threshold", ctypes.c_float),
                ("spawn_number_change_rate", ctypes.c_float), ("mutation", TnMutationParams)]


class TnSpeciesTable(ctypes.Structure):
    _fields_ = [("max_species", ctypes.c_int32), ("reps", TnPopulationArrays),
                ("alive", c_int32_p), ("best", c_float_p), ("last_improved", c_int32_p),
                ("size", c_int32_p)]


class TnBucketInfo(ctypes.Structure):
    _fields_ = [("engine", ctypes.c_int32), ("rows_class", ctypes.c_int32),
                ("count", ctypes.c_int32), ("edges", ctypes.c_int64), ("tile", TnTile)]


_POP = ctypes.POINTER(TnPopulation)
_TR = ctypes.POINTER(TnTransformed)
_STREAM = ctypes.c_void_p

# name -> (restype, argtypes)
SIGNATURES = {
    "tn_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "tn_version": (ctypes.c_int, []),
    "tn_last_error": (ctypes.c_char_p, []),
    "tn_validate_population": (ctypes.c_int, [_POP]),
    "tn_transformed_size": (ctypes.c_int, [_POP, ctypes.POINTER(TnTransformedElems)]),
    "tn_transform": (ctypes.c_int, [_POP, _TR, _STREAM]),
    "tn_pack_paper_layout": (ctypes.c_int, [c_float_p, c_float_p, ctypes.c_int32, ctypes.c_int32,
                                            ctypes.c_int32, ctypes.POINTER(TnPopulationArrays),
                                            c_int32_p, _STREAM]),
    "tn_forward": (ctypes.c_int, [_POP, _TR, c_float_p, ctypes.c_int64, ctypes.c_int32,
                                  c_float_p, _STREAM]),
    "tn_forward_tiled": (ctypes.c_int, [_POP, _TR, c_float_p, ctypes.c_int64, ctypes.c_int32,
                                        c_float_p, ctypes.POINTER(TnTile), _STREAM]),
    "tn_forward_loss": (ctypes.c_int, [_POP, _TR, c_float_p, ctypes.c_int64, ctypes.c_int32,
                                       c_float_p, ctypes.c_int64, ctypes.c_float,
                                       ctypes.c_float, c_float_p, c_float_p, _STREAM]),
    "tn_backward": (ctypes.c_int, [_POP, _TR, c_float_p, ctypes.c_int64, ctypes.c_int32,
                                   c_float_p, ctypes.c_int64, c_float_p, c_float_p, _STREAM]),
    "tn_forward_backward_mse": (ctypes.c_int, [_POP, _TR, c_float_p, ctypes.c_int64,
                                               ctypes.c_int32, c_float_p, ctypes.c_int64,
                                               c_float_p, c_float_p, c_float_p, _STREAM]),
    "tn_distance_workspace_size": (ctypes.c_int, [_POP, ctypes.POINTER(ctypes.c_size_t)]),
    "tn_distance": (ctypes.c_int, [_POP, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                   ctypes.c_void_p, c_float_p, c_int32_p, c_int32_p, _STREAM]),
    "tn_distance_noalloc": (ctypes.c_int, [_POP, ctypes.c_float, ctypes.c_float,
                                           ctypes.c_float, c_float_p, c_int32_p, c_int32_p,
                                           _STREAM]),
    "tn_distance_nodes_workspace_size": (ctypes.c_int, [_POP, ctypes.POINTER(ctypes.c_size_t)]),
    "tn_distance_nodes": (ctypes.c_int, [_POP, ctypes.c_float, ctypes.c_float, ctypes.c_void_p,
                                         c_float_p, c_int32_p, c_int32_p, _STREAM]),
    "tn_reproduce_draws": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, c_int32_p, c_int32_p]),
    "tn_reproduce_workspace_size": (ctypes.c_int, [ctypes.c_int32,
                                                   ctypes.POINTER(ctypes.c_size_t)]),
    "tn_reproduce": (ctypes.c_int, [_POP, ctypes.c_int32, c_int32_p, c_float_p, c_float_p,
                                    ctypes.POINTER(TnMutationParams), ctypes.c_int32,
                                    ctypes.POINTER(TnPopulationArrays), c_int32_p,
                                    ctypes.c_void_p, _STREAM]),
    "tn_forward_recurrent": (ctypes.c_int, [_POP, c_float_p, ctypes.c_int64, ctypes.c_int32,
                                            ctypes.c_int32, c_float_p, c_int32_p, _STREAM]),
    "tn_neat_init": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                    ctypes.c_int32, c_float_p, ctypes.POINTER(TnMutationParams),
                                    ctypes.POINTER(TnPopulationArrays),
                                    ctypes.POINTER(TnSpeciesTable), _STREAM]),
    "tn_neat_workspace_size": (ctypes.c_int, [_POP, ctypes.c_int32,
                                              ctypes.POINTER(ctypes.c_size_t)]),
    "tn_neat_generation": (ctypes.c_int, [_POP, c_float_p, ctypes.c_int32,
                                          ctypes.POINTER(TnNeatParams),
                                          ctypes.POINTER(TnSpeciesTable), c_float_p, c_float_p,
                                          c_float_p, ctypes.c_int32,
                                          ctypes.POINTER(TnPopulationArrays), c_int32_p,
                                          c_int32_p, c_int32_p, ctypes.c_void_p, _STREAM]),
    "tn_plan_create": (ctypes.c_int, [_POP, _TR, ctypes.c_int32, ctypes.c_char_p,
                                      ctypes.POINTER(ctypes.c_void_p), _STREAM]),
    "tn_plan_destroy": (None, [ctypes.c_void_p]),
    "tn_plan_num_buckets": (ctypes.c_int, [ctypes.c_void_p]),
    "tn_plan_bucket": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32,
                                      ctypes.POINTER(TnBucketInfo)]),
    "tn_plan_set_tile": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                        ctypes.c_int32]),
    "tn_plan_forward": (ctypes.c_int, [ctypes.c_void_p, c_float_p, ctypes.c_int64, c_float_p,
                                       _STREAM]),
    "tn_plan_forward_buckets": (ctypes.c_int, [ctypes.c_void_p, c_float_p, ctypes.c_int64,
                                               c_float_p, _STREAM]),
    "tn_plan_tune": (ctypes.c_int, [ctypes.c_void_p, c_float_p, ctypes.c_int64, c_float_p,
                                    ctypes.c_char_p, _STREAM]),
    "tn_plan_forward_bucket": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                              c_float_p, ctypes.c_int64, c_float_p, _STREAM]),
    "tn_cppn_query": (ctypes.c_int, [_POP, _TR, ctypes.POINTER(TnSubstrate), ctypes.c_void_p,
                                     ctypes.c_void_p, c_float_p, c_float_p, _STREAM]),
    "tn_substrate_workspace_size": (ctypes.c_int, [ctypes.POINTER(TnSubstrate), ctypes.c_int32,
                                                   ctypes.c_int32, ctypes.c_int64,
                                                   ctypes.POINTER(ctypes.c_size_t)]),
    "tn_substrate_backward": (ctypes.c_int, [ctypes.POINTER(TnSubstrate), ctypes.c_int32,
                                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                             ctypes.c_int32, c_float_p, c_float_p,
                                             ctypes.c_void_p, c_float_p, c_float_p, _STREAM]),
    "tn_cppn_backward_workspace_size": (ctypes.c_int, [_POP, ctypes.POINTER(TnSubstrate),
                                                       ctypes.POINTER(ctypes.c_size_t)]),
    "tn_cppn_backward": (ctypes.c_int, [_POP, _TR, ctypes.POINTER(TnSubstrate), c_float_p,
                                        c_float_p, ctypes.c_void_p, c_float_p, c_float_p,
                                        _STREAM]),
    "tn_substrate_forward": (ctypes.c_int, [ctypes.POINTER(TnSubstrate), ctypes.c_int32,
                                            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.c_int64, ctypes.c_int32, c_float_p, c_float_p,
                                            _STREAM]),
}


def load(path: str = LIB_PATH):
    if not os.path.exists(path):
        raise ImportError(
            f"libtnhip.so not found at {path}; build it with "
            "`python -c 'import __graft_entry__ as g; g.build()'` "
            "(or python paper_2504_08339_amd/build.py)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


class TNError(RuntimeError):
    def __init__(self, call: str, code: int, text: str):
        super().__init__(f"{call} failed: {text} ({code})")
        self.code = code
