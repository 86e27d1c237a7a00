"""Seeded synthetic inputs for the population-evaluation path.

This package only *generates* inputs: padded or ragged structure-of-arrays
populations of NEAT genomes, observation batches and regression targets. It
holds none of the method's arithmetic (no topological sort, no forward pass,
no distance); both the HIP library's tests/bench and the CPU oracle read what
it writes.
"""
from .population import (  # noqa: F401
    ACT, AGG, Population, grow_population, random_dag_population,
    xor_population, control_population, batching_population,
    differentiation_population, cppn_population, permute_rows, insert_holes,
    to_ragged, to_padded, subset, xor_inputs, xor_targets, normal_obs,
    uniform_inputs, target_mlp, CONFIG_SEEDS, to_paper_layout,
    reproduction_draws, recurrent_population,
)
