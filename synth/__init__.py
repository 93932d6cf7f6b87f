"""Seeded synthetic hypergraph inputs shared by the oracle side and the GPU side.

This package holds input generation only: hyperedge sizes, member sets,
hyperedge weights, coarsest-level embeddings, labels, cotangents and
bag-of-words node features.  It
contains none of the refinement method's arithmetic (no coarsening, no
projection, no sweep), so both the FP64 oracle and the HIP path can take
their inputs from it without sharing any of the method.
"""
from .hypergraph import (  # noqa: F401
    CONFIGS,
    Config,
    Hypergraph,
    bag_of_words,
    make_hypergraph,
    node_features,
    coarsest_embedding,
    drop_isolated_and_singletons,
    labelled_nodes,
    linear_head,
    cotangent,
    random_hypergraph,
)
