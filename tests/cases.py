"""Shared input builders for the parity tests: the same seeded hypergraph goes
to the oracle (its own hierarchy) and to the library (its own hierarchy);
the two hierarchies are compared bit for bit before any embedding is."""
import numpy as np

from synth import CONFIGS, coarsest_embedding, make_hypergraph, random_hypergraph


def rel_fro(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def max_abs_rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)) if b.size else 0.0


def both_hierarchies(O, H, hg, n_coarsen):
    """(oracle levels, oracle maps, library Hierarchy), checked identical."""
    levels, maps = O.build_hierarchy(hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, hg.edge_w, n_coarsen)
    hier = H.Hierarchy.build(hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, hg.edge_w, n_coarsen)
    for a, b in zip(hier.levels, levels):
        assert a.n_nodes == b.n_nodes and a.n_edges == b.n_edges
        assert np.array_equal(a.edge_ptr, b.eptr) and np.array_equal(a.edge_idx, b.eidx)
    for a, b in zip(hier.maps, maps):
        assert np.array_equal(a.node_rep, b.node_rep) and np.array_equal(a.edge_rep, b.edge_rep)
    return levels, maps, hier


def tier_hypergraph(seed, small_max, chunk):
    """A hypergraph whose rows land on every tier boundary: hyperedges of
    size 1, small_max, small_max + 1, chunk, chunk + 1, several chunks, and
    nodes of degree 0, 1, small_max, small_max + 1, chunk + 1 and a hub."""
    rng = np.random.default_rng(seed)
    n_nodes = 4 * chunk + 64
    sizes = [1, 2, small_max, small_max + 1, chunk, chunk + 1, 3 * chunk + 5, max(1, small_max - 1)]
    sizes += list(rng.integers(1, small_max + 3, size=40))
    edges = [sorted(rng.choice(n_nodes - 8, size=s, replace=False).tolist()) for s in sizes]
    # a hub node in many hyperedges, a node with exactly small_max + 1, one
    # with small_max and one isolated (n_nodes - 1 never used)
    hub, a, b = n_nodes - 2, n_nodes - 3, n_nodes - 4
    deg_wanted = {hub: 2 * chunk + 7, a: small_max + 1, b: small_max}
    for node, k in deg_wanted.items():
        for _ in range(k):
            edges.append([node])
        # and membership in some bigger hyperedges too
        for e in rng.choice(len(sizes), size=3, replace=False):
            if node not in edges[e]:
                edges[e] = sorted(edges[e] + [node])
    ptr = np.concatenate([[0], np.cumsum([len(e) for e in edges])]).astype(np.int64)
    idx = np.array([v for e in edges for v in e], dtype=np.int32)
    w = rng.uniform(0.5, 2.0, size=len(edges)).astype(np.float32)
    from synth.hypergraph import Hypergraph
    return Hypergraph(n_nodes, len(edges), ptr, idx, w)


__all__ = ["CONFIGS", "coarsest_embedding", "make_hypergraph", "random_hypergraph", "rel_fro", "max_abs_rel",
           "both_hierarchies", "tier_hypergraph"]
