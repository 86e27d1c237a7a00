"""CPU oracle for tensorized NEAT population evaluation.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import or call this
package: only the test-suite, the smoke check and the benchmark's CPU-baseline
leg use it. It shares no code with the HIP library (kernels, headers, helpers or
tables) and reads only the seeded synthetic inputs.

It is the plain, slow definition of what the method computes, in float64
(the paper fixes no precision), following TensorNEAT (arXiv 2504.08339):

* ``genome``   - decoding the padded node/connection tensors (Section 3.1) and
                 the feedforward transformation: topological order plus the
                 expanded connections as per-node in-edge lists (Section 3.3).
* ``inference`` - the calculation stage (Section 3.3): node values in
                 topological order, f_c = w * input, f_n = act(agg(.) + b),
                 plus the XOR fitness and MSE loss epilogues.
* ``compat``   - the speciation compatibility distance over connection genes
                 aligned by historical marking (Section 2.1, Appendix A), and
                 the node-inclusive form with the paper's coefficient pair.
* ``adjoint``  - reverse-mode derivative of the calculation stage with respect
                 to connection weights and node biases.
* ``hyperneat``- CPPN queries over a grid substrate and the substrate forward
                 (HyperNEAT, named in Section 4.4).
* ``recurrent`` - forward pass of recurrent networks by synchronous sweeps
                 (network type of Appendix A; Section 3.3 covers only the
                 feedforward calculation).
* ``neat``     - one NEAT generation (Algorithm 1's loop body: speciation,
                 offspring counts, parent selection, reproduction) and the
                 initial population.
* ``reproduce`` - crossover and mutation as tensorized row operations
                 (Section 3.2; hyperparameters of Appendices A and C).

Every place where the paper is silent takes one stated reading; each function's
docstring names it.
"""
from .genome import (  # noqa: F401
    CYCLE, DANGLING, DUP_CONN, DUP_NODE, INPUT_DST, MISSING_IO, OVERSIZE, BAD_ATTR,
    ACT_NAMES, AGG_NAMES, Genome, Transformed, decode, transform,
    transform_population, transform_arrays,
)
from .inference import (  # noqa: F401
    activate, activation_slope, aggregate, forward, forward_population,
    xor_fitness, sse_loss,
)
from .compat import (  # noqa: F401
    genome_genes, distance, distance_matrix, node_genes, distance_nodes, distance_nodes_matrix,
)
from .adjoint import backward, backward_population  # noqa: F401
from . import hyperneat  # noqa: F401
from . import reproduce  # noqa: F401
from . import neat  # noqa: F401
from .recurrent import recurrent_forward, recurrent_population, recurrent_status  # noqa: F401
