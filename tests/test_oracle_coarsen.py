"""Pins for the oracle's coarsening (Section 3.1, Algorithm 1, featureless):
an independent brute-force re-derivation with Python sets on small random
hypergraphs, and invariants that any correct contraction satisfies."""
import numpy as np
import pytest

from synth import CONFIGS, make_hypergraph, random_hypergraph


def brute_force_coarsen(n_nodes, edges, w):
    """edges: list of member sets; w: list of weights.  Re-derives the whole
    contraction from the rules: assignment by (weight desc, size asc, id asc),
    groups numbered by smallest member, removal of fully-assigned hyperedges,
    coarse member sets through rep()."""
    inc = {v: [e for e, m in enumerate(edges) if v in m] for v in range(n_nodes)}
    choice = {}
    for v in range(n_nodes):
        if inc[v]:
            choice[v] = min(inc[v], key=lambda e: (-w[e], len(edges[e]), e))
    groups = {}
    for v in range(n_nodes):
        key = ("e", choice[v]) if v in choice else ("v", v)
        groups.setdefault(key, []).append(v)
    ordered = sorted(groups.values(), key=min)
    rep = {}
    for gid, members in enumerate(ordered):
        for v in members:
            rep[v] = gid
    edge_rep, coarse_edges, coarse_w = [], [], []
    for e, m in enumerate(edges):
        if all(choice.get(v) == e for v in m):
            edge_rep.append(-1)
        else:
            edge_rep.append(len(coarse_edges))
            coarse_edges.append(sorted({rep[v] for v in m}))
            coarse_w.append(w[e])
    return [rep[v] for v in range(n_nodes)], edge_rep, len(ordered), coarse_edges, coarse_w


def _edges(hg):
    return [set(int(v) for v in hg.edge_idx[hg.edge_ptr[e]:hg.edge_ptr[e + 1]]) for e in range(hg.n_edges)]


@pytest.mark.parametrize("seed", range(40))
def test_coarsen_matches_brute_force(oracle_mod, seed):
    O = oracle_mod
    hg = random_hypergraph(seed, 6 + seed % 25, 3 + seed % 17, 1, 6, weighted=(seed % 3 != 0),
                           integer_weights=(seed % 3 == 1))
    lv = O.Level(hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, hg.edge_w)
    c = O.coarsen_level(lv)
    w = [1.0] * hg.n_edges if hg.edge_w is None else [float(x) for x in hg.edge_w]
    rep, erep, nvc, cedges, cw = brute_force_coarsen(hg.n_nodes, _edges(hg), w)
    assert list(c.node_rep) == rep
    assert list(c.edge_rep) == erep
    assert c.coarse.n_nodes == nvc and c.coarse.n_edges == len(cedges)
    got = [list(c.coarse.eidx[c.coarse.eptr[e]:c.coarse.eptr[e + 1]]) for e in range(c.coarse.n_edges)]
    assert got == cedges
    if hg.edge_w is not None:
        assert list(c.coarse.w) == [np.float32(x) for x in cw]


def _check_invariants(O, lv, c):
    node_rep, edge_rep, co = c.node_rep, c.edge_rep, c.coarse
    # preimages of the coarse nodes partition V
    assert node_rep.min() >= 0 and node_rep.max() == co.n_nodes - 1
    assert len(np.unique(node_rep)) == co.n_nodes
    # each group of two or more nodes lies inside one fine hyperedge, and
    # groups are numbered by their smallest member
    first = np.full(co.n_nodes, -1)
    for v in range(lv.n_nodes):
        if first[node_rep[v]] < 0:
            first[node_rep[v]] = v
    assert np.all(np.diff(first) > 0)
    incident = [set() for _ in range(lv.n_nodes)]
    for e in range(lv.n_edges):
        for v in lv.eidx[lv.eptr[e]:lv.eptr[e + 1]]:
            incident[v].add(e)
    groups = {}
    for v in range(lv.n_nodes):
        groups.setdefault(int(node_rep[v]), []).append(v)
    for members in groups.values():
        if len(members) > 1:
            assert set.intersection(*(incident[v] for v in members))
    # kept hyperedges keep their relative order; removed ones are fully merged
    kept = edge_rep[edge_rep >= 0]
    assert np.array_equal(kept, np.arange(co.n_edges))
    for e in np.nonzero(edge_rep < 0)[0]:
        members = lv.eidx[lv.eptr[e]:lv.eptr[e + 1]]
        assert len(np.unique(node_rep[members])) == 1
    assert co.nnz <= lv.nnz and co.n_edges <= lv.n_edges and co.n_nodes <= lv.n_nodes
    for e in range(co.n_edges):
        row = co.eidx[co.eptr[e]:co.eptr[e + 1]]
        assert len(row) >= 1 and np.all(np.diff(row) > 0)


@pytest.mark.parametrize("seed", range(8))
def test_coarsen_invariants_random(oracle_mod, seed):
    O = oracle_mod
    hg = random_hypergraph(100 + seed, 300, 200, 1, 9, weighted=bool(seed % 2))
    lv = O.Level(hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, hg.edge_w)
    for _ in range(3):
        c = O.coarsen_level(lv)
        _check_invariants(O, lv, c)
        lv = c.coarse


def test_coarsen_invariants_c1(oracle_mod):
    O = oracle_mod
    cfg = CONFIGS["tiny-2k"]
    hg = make_hypergraph(cfg)
    levels, maps = O.build_hierarchy(hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, hg.edge_w, cfg.levels)
    for lvl, c in enumerate(maps):
        _check_invariants(O, levels[lvl], c)
    sizes = [(lv.n_nodes, lv.n_edges, lv.nnz) for lv in levels]
    assert all(a >= b for a, b in zip(sizes, sizes[1:]))


def test_projection_rows_and_removed_hyperedges(oracle_mod):
    """A removed hyperedge's projected row equals the mean of its members'
    projected rows (all members went to one coarse node)."""
    O = oracle_mod
    hg = random_hypergraph(5, 200, 150, 2, 6, weighted=False)
    lv = O.Level(hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, None)
    c = O.coarsen_level(lv)
    rm = O.rowmap(lv, c)
    zc = np.random.default_rng(2).standard_normal((c.coarse.rows, 4))
    zf = O.project(rm, zc)
    np.testing.assert_array_equal(zf, zc[rm])
    assert np.any(c.edge_rep < 0)
    for e in np.nonzero(c.edge_rep < 0)[0]:
        members = lv.eidx[lv.eptr[e]:lv.eptr[e + 1]]
        np.testing.assert_allclose(zf[lv.n_nodes + e], zf[members].mean(axis=0), atol=1e-14)
    for e in np.nonzero(c.edge_rep >= 0)[0]:
        np.testing.assert_array_equal(zf[lv.n_nodes + e], zc[c.coarse.n_nodes + c.edge_rep[e]])
