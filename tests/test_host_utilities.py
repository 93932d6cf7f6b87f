"""Host utilities around the hot path: the star-expansion edge list handed
to an initial embedder (Section 1.1, Section 3.2), the optional depth rule
of the coarsening (Section 3.1), and the dataset cleaning of Section 4."""
import numpy as np
import pytest

from synth import drop_isolated_and_singletons, random_hypergraph
from synth.hypergraph import Hypergraph


@pytest.fixture(scope="module")
def H():
    import paper_2103_09660_amd as H
    H.abi_version()
    return H


def test_star_edgelist_small_example(H):
    # nodes 0..3, e0 = {0,1,2} (w 2), e1 = {2,3} (w 0.5): rows 4 and 5
    lv = H.HostLevel(4, 2, np.array([0, 3, 5]), np.array([0, 1, 2, 2, 3]), np.array([2.0, 0.5], np.float32))
    src, dst, w = H.star_edgelist(lv)
    assert src.tolist() == [0, 1, 2, 2, 3]
    assert dst.tolist() == [4, 4, 4, 5, 5]
    assert w.tolist() == [2.0, 2.0, 2.0, 0.5, 0.5]
    src, dst, w = H.star_edgelist(H.HostLevel(4, 2, np.array([0, 3, 5]), np.array([0, 1, 2, 2, 3]), None))
    assert w.tolist() == [1.0] * 5


def test_star_edgelist_matches_the_incidence(H):
    hg = random_hypergraph(3, 500, 300, 1, 9)
    hier = H.Hierarchy.build(hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, hg.edge_w, 3)
    c = hier.levels[-1]
    src, dst, w = hier.coarsest_edgelist()
    assert len(src) == c.nnz and src.max() < c.n_nodes and dst.min() >= c.n_nodes and dst.max() < c.rows
    # every (node, hyperedge) pair appears once, as in the member lists
    pairs = set(zip(src.tolist(), (dst - c.n_nodes).tolist()))
    ref = {(int(v), e) for e in range(c.n_edges) for v in c.edge_idx[c.edge_ptr[e]:c.edge_ptr[e + 1]]}
    assert pairs == ref and len(pairs) == c.nnz
    assert np.array_equal(w, np.repeat(c.edge_w, np.diff(c.edge_ptr)))


def test_depth_rule(H):
    hg = random_hypergraph(5, 3000, 2000, 1, 6)
    full = H.Hierarchy.build(hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, hg.edge_w, 6)
    assert full.n_levels == 7
    rows = [lv.rows for lv in full.levels]
    # stop once a level has at most min_rows rows: the first such level is the coarsest
    target = rows[3]
    cut = H.Hierarchy.build(hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, hg.edge_w, 6, min_rows=target)
    assert cut.n_levels == 4 and cut.levels[-1].rows == target
    for a, b in zip(cut.maps, full.maps):
        assert np.array_equal(a.node_rep, b.node_rep) and np.array_equal(a.edge_rep, b.edge_rep)
    # a level that no longer shrinks stops the coarsening (nodes only: nothing merges)
    iso = H.Hierarchy.build(5, 0, np.zeros(1, np.int64), np.zeros(0, np.int32), None, 4, min_rows=1)
    assert iso.n_levels == 1
    # min_rows = 0 keeps the fixed depth, even when steps stall
    fixed = H.Hierarchy.build(5, 0, np.zeros(1, np.int64), np.zeros(0, np.int32), None, 3)
    assert fixed.n_levels == 4


def test_drop_isolated_and_singletons():
    # nodes 0..6; e0 = {1} (singleton), e1 = {0,2,5}, e2 = {3}, e3 = {2,5}; nodes 1, 3, 4, 6 end up unused
    hg = Hypergraph(7, 4, np.array([0, 1, 4, 5, 7]), np.array([1, 0, 2, 5, 3, 2, 5], np.int32),
                    np.array([1.0, 2.0, 3.0, 4.0], np.float32))
    p, kept = drop_isolated_and_singletons(hg)
    assert kept.tolist() == [0, 2, 5]
    assert (p.n_nodes, p.n_edges) == (3, 2)
    assert p.edge_ptr.tolist() == [0, 3, 5] and p.edge_idx.tolist() == [0, 1, 2, 1, 2]
    assert p.edge_w.tolist() == [2.0, 4.0]
    big = random_hypergraph(9, 2000, 1500, 1, 6)
    q, kept = drop_isolated_and_singletons(big)
    assert np.diff(q.edge_ptr).min() >= 2
    assert len(np.unique(q.edge_idx)) == q.n_nodes
    # renumbered rows stay ascending and map back to the input members
    for e in range(0, q.n_edges, 97):
        row = q.edge_idx[q.edge_ptr[e]:q.edge_ptr[e + 1]]
        assert np.all(np.diff(row) > 0)
