"""Pins for the oracle's coarsening with node features (Section 3.1,
Algorithm 1 with X): a hand-worked example, a brute-force re-derivation with
exact rational cosines, the special cases that reduce to the featureless
rule, and the conservation of the feature mass in X'."""
from fractions import Fraction

import numpy as np
import pytest

from synth import random_hypergraph
from synth.hypergraph import bag_of_words
from tests.golden_io import read_fixture


def _edges(hg):
    return [[int(v) for v in hg.edge_idx[hg.edge_ptr[e]:hg.edge_ptr[e + 1]]] for e in range(hg.n_edges)]


def brute_force_features(n_nodes, edges, w, x):
    """Re-derives the maps and X' from the rules with exact arithmetic:
    f(e) is the mean of member rows as a Fraction vector, cos^2 with its sign
    is compared as a Fraction, equal cosines go to the featureless order
    (weight desc, size asc, id asc); a cosine with a zero vector counts as 0."""
    k = x.shape[1]
    feats = [[Fraction(sum(int(x[v, j]) for v in m), len(m)) for j in range(k)] for m in edges]

    def cos_key(e, v):
        fe, fv = feats[e], [int(t) for t in x[v]]
        d = sum(a * b for a, b in zip(fe, fv))
        ne = sum(a * a for a in fe)
        nv = sum(b * b for b in fv)
        if ne == 0 or nv == 0:
            return Fraction(0)
        c2 = d * d / (ne * nv)
        return c2 if d >= 0 else -c2

    choice = {}
    for v in range(n_nodes):
        inc = [e for e, m in enumerate(edges) if v in m]
        if inc:
            choice[v] = min(inc, key=lambda e: (-cos_key(e, v), -w[e], len(edges[e]), e))
    groups = {}
    for v in range(n_nodes):
        groups.setdefault(("e", choice[v]) if v in choice else ("v", v), []).append(v)
    ordered = sorted(groups.values(), key=min)
    rep = {v: g for g, members in enumerate(ordered) for v in members}
    edge_rep, coarse = [], []
    for e, m in enumerate(edges):
        if all(choice.get(v) == e for v in m):
            edge_rep.append(-1)
        else:
            edge_rep.append(len(coarse))
            coarse.append(sorted({rep[v] for v in m}))
    xc = np.zeros((len(ordered), k), dtype=np.int64)
    for v in range(n_nodes):
        xc[rep[v]] += x[v]
    return [rep[v] for v in range(n_nodes)], edge_rep, coarse, xc


def _run(O, hg, x):
    lv = O.Level(hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, hg.edge_w)
    return O.coarsen_level_features(lv, x)


def _check(c, xc, expect):
    rep, erep, coarse, xref = expect
    assert c.node_rep.tolist() == rep
    assert c.edge_rep.tolist() == erep
    got = [c.coarse.eidx[c.coarse.eptr[i]:c.coarse.eptr[i + 1]].tolist() for i in range(c.coarse.n_edges)]
    assert got == coarse
    assert np.array_equal(xc.astype(np.int64), xref)


def test_hand_worked_example(oracle_mod):
    from synth.hypergraph import Hypergraph
    g = read_fixture("features_example.txt")
    n = int(g["n_nodes"][0][0])
    edges = [[int(v) for v in row] for row in g["edge"]]
    ptr = np.concatenate([[0], np.cumsum([len(m) for m in edges])]).astype(np.int64)
    hg = Hypergraph(n, len(edges), ptr, np.concatenate(edges).astype(np.int32), None)
    x = np.array([[int(v) for v in row] for row in g["x"]], dtype=np.int32)
    c, xc = _run(oracle_mod, hg, x)
    assert c.node_rep.tolist() == [int(v) for v in g["node_rep"][0]]
    assert c.edge_rep.tolist() == [int(v) for v in g["edge_rep"][0]]
    coarse = [c.coarse.eidx[c.coarse.eptr[i]:c.coarse.eptr[i + 1]].tolist() for i in range(c.coarse.n_edges)]
    assert coarse == [[int(v) for v in row] for row in g["coarse_edge"]]
    assert xc.tolist() == [[int(v) for v in row] for row in g["coarse_x"]]


@pytest.mark.parametrize("seed", range(30))
def test_matches_exact_brute_force(oracle_mod, seed):
    hg = random_hypergraph(seed, 8 + seed % 23, 4 + seed % 19, 1, 6, weighted=(seed % 3 != 0),
                           integer_weights=(seed % 3 == 1))
    k = 4 * (1 + seed % 3)
    x = bag_of_words(1000 + seed, hg.n_nodes, k, 1, min(4, k), max_count=3, empty_frac=0.1, repeat_frac=0.3)
    w = [1.0] * hg.n_edges if hg.edge_w is None else [float(v) for v in hg.edge_w]
    c, xc = _run(oracle_mod, hg, x)
    _check(c, xc, brute_force_features(hg.n_nodes, _edges(hg), w, x))


@pytest.mark.parametrize("seed", range(6))
def test_zero_or_identical_features_reduce_to_featureless(oracle_mod, seed):
    """All cosines equal (every row zero, or every row the same nonzero
    document): the featureless order decides alone."""
    O = oracle_mod
    hg = random_hypergraph(50 + seed, 300, 200, 1, 7, weighted=(seed % 2 == 0), integer_weights=True)
    lv = O.Level(hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, hg.edge_w)
    ref = O.coarsen_level(lv)
    for x in (np.zeros((hg.n_nodes, 8), dtype=np.int32),
              np.tile(np.array([[2, 0, 1, 0, 0, 3, 0, 1]], dtype=np.int32), (hg.n_nodes, 1))):
        c, xc = O.coarsen_level_features(lv, x)
        assert np.array_equal(c.node_rep, ref.node_rep) and np.array_equal(c.edge_rep, ref.edge_rep)
        assert np.array_equal(c.coarse.eidx, ref.coarse.eidx)
        assert np.array_equal(xc.sum(axis=0), x.sum(axis=0))


def test_feature_mass_and_group_sums(oracle_mod):
    """X' keeps every column total and each row is the sum over its group."""
    O = oracle_mod
    hg = random_hypergraph(7, 3000, 2000, 1, 9)
    x = bag_of_words(7, hg.n_nodes, 64, 3, 12)
    c, xc = _run(O, hg, x)
    assert np.array_equal(xc.sum(axis=0), x.sum(axis=0))
    ref = np.zeros_like(xc)
    np.add.at(ref, c.node_rep, x)
    assert np.array_equal(ref, xc)
    assert xc.shape[0] == c.coarse.n_nodes


def test_features_change_the_choice(oracle_mod):
    """Features matter: on a random workload a large share of the nodes with
    two or more hyperedges choose differently than without features."""
    O = oracle_mod
    hg = random_hypergraph(9, 2000, 1500, 2, 8)
    lv = O.Level(hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, hg.edge_w)
    x = bag_of_words(9, hg.n_nodes, 128, 5, 20)
    c, _ = O.coarsen_level_features(lv, x)
    ref = O.coarsen_level(lv)
    assert not np.array_equal(c.node_rep, ref.node_rep)
