"""StaticGreedy influence maximisation on one MI355X (gfx950).

Cheng et al., "StaticGreedy: Solving the Scalability-Accuracy Dilemma in
Influence Maximization", CIKM 2013 (arXiv 1212.4779). The selection runs in
hand-written HIP kernels behind the C ABI of include/im.h; this package only
passes torch tensors' device pointers and the current stream to it.
"""
from ._native import ImError  # noqa: F401
from .api import (Workspace, Graph, Plan, BatchPlan, Mlp, select, select_batch, select_lazy,  # noqa: F401
                  initial_gains, snapshot_masks, transpose, validate, node_features,
                  mlp_samples, autotune, autotune_batch, spread,
                  pair_ids, select_undirected, select_noalloc, autotune_lazy)
