"""MI355X-native tensorized NEAT population evaluation (TensorNEAT, arXiv 2504.08339).

The computation lives in libtnhip.so (HIP for gfx950, C ABI in
include/tensorneat_hip.h); this package marshals torch tensors to it. Importing
the package loads the library and fails loudly if it has not been built.
"""
from ._abi import (  # noqa: F401
    TNError, TN_CYCLE, TN_DANGLING, TN_DUP_CONN, TN_DUP_NODE, TN_INPUT_DST, TN_MISSING_IO,
    TN_OVERSIZE, TN_BAD_ATTR, TN_MAX_NODES, TN_MAX_CONNS, TN_ENGINE_AUTO, TN_ENGINE_LDS,
    TN_ENGINE_REG, TN_PACK_NODE_KEY, TN_PACK_NODE_CODE, TN_PACK_CONN_KEY, TN_PACK_CONN_FLAG,
)
from .api import (  # noqa: F401
    Population, Transformed, DistanceWorkspace, transform, forward, forward_loss, distance, lib,
    backward, forward_backward_mse, Plan, cppn_query, substrate_forward,
    substrate_backward, cppn_backward, pack_paper_layout, distance_noalloc, distance_nodes,
    MutationParams, reproduce, reproduce_draws, forward_recurrent,
    NeatParams, SpeciesTable, neat_init, neat_generation,
)
from .autograd import TNForward  # noqa: F401
