"""Pins for the oracle's sweep, projection and multi-level loop against the
paper's matrix statement and against closed forms and invariants that the
mathematics fixes (Section 3.3, Algorithm 2)."""
import numpy as np
import pytest
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import connected_components

from synth import random_hypergraph
from tests.dense_ref import edge_first_matrix, jacobi_matrix, projection_matrix, star_adjacency

SEEDS = [0, 1, 2, 3, 4, 5]


def _level(O, hg):
    return O.Level(hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, hg.edge_w)


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("seed", SEEDS)
@pytest.mark.parametrize("omega", [0.5, 0.3, 1.0])
def test_sweep_equals_dense_laplacian_form(oracle_mod, seed, omega):
    O = oracle_mod
    hg = random_hypergraph(seed, 37, 23, 1, 6, weighted=(seed % 2 == 0))
    lv = _level(O, hg)
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((lv.rows, 3))
    A = star_adjacency(hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, hg.edge_w)
    assert _rel(O.sweep(lv, z, omega, 0), jacobi_matrix(A, omega) @ z) < 1e-13
    assert _rel(O.sweep(lv, z, omega, 1), edge_first_matrix(A, omega, hg.n_nodes) @ z) < 1e-13


def test_single_hyperedge_closed_form(oracle_mod):
    """One hyperedge of n members, Jacobi: with m0 the member mean and e0 the
    hyperedge row, e_i = (m0+e0)/2 + (1-2w)^i (e0-m0)/2 and
    z_u,i = (m0+e0)/2 - (1-2w)^i (e0-m0)/2 + (1-w)^i (z_u,0 - m0)."""
    O = oracle_mod
    n = 7
    lv = O.Level(n, 1, np.array([0, n]), np.arange(n, dtype=np.int32), None)
    rng = np.random.default_rng(11)
    z0 = rng.standard_normal((n + 1, 2))
    for w in (0.5, 0.25, 0.8):
        z = z0.copy()
        m0 = z0[:n].mean(axis=0)
        e0 = z0[n]
        for i in range(1, 9):
            z = O.sweep(lv, z, w, 0)
            e_i = (m0 + e0) / 2 + (1 - 2 * w) ** i * (e0 - m0) / 2
            zu = (m0 + e0) / 2 - (1 - 2 * w) ** i * (e0 - m0) / 2 + (1 - w) ** i * (z0[:n] - m0)
            np.testing.assert_allclose(z[n], e_i, rtol=0, atol=1e-13)
            np.testing.assert_allclose(z[:n], zu, rtol=0, atol=1e-13)


def _components(hg):
    R = hg.n_nodes + hg.n_edges
    rows, cols = [], []
    for e in range(hg.n_edges):
        for j in range(hg.edge_ptr[e], hg.edge_ptr[e + 1]):
            rows.append(int(hg.edge_idx[j]))
            cols.append(hg.n_nodes + e)
    g = csr_matrix((np.ones(len(rows)), (rows, cols)), shape=(R, R))
    return connected_components(g, directed=False)[1]


def _pi(hg):
    """Stationary weights of the averaging: weighted degree of each row."""
    w = np.ones(hg.n_edges) if hg.edge_w is None else hg.edge_w.astype(np.float64)
    pi = np.zeros(hg.n_nodes + hg.n_edges)
    sizes = np.diff(hg.edge_ptr)
    for e in range(hg.n_edges):
        pi[hg.n_nodes + e] = sizes[e] * w[e]
        for j in range(hg.edge_ptr[e], hg.edge_ptr[e + 1]):
            pi[hg.edge_idx[j]] += w[e]
    return pi


@pytest.mark.parametrize("seed", SEEDS)
def test_constant_per_component_is_fixed_point(oracle_mod, seed):
    O = oracle_mod
    hg = random_hypergraph(seed, 50, 20, 1, 4)
    lv = _level(O, hg)
    comp = _components(hg)
    z = np.stack([comp * 1.5 - 2.0, np.full(lv.rows, 3.25)], axis=1)
    for order in (0, 1):
        out = z
        for _ in range(5):
            out = O.sweep(lv, out, 0.5, order)
        np.testing.assert_allclose(out, z, rtol=0, atol=1e-13)


@pytest.mark.parametrize("seed", SEEDS)
def test_jacobi_conserves_pi_weighted_sum_edge_first_does_not(oracle_mod, seed):
    O = oracle_mod
    hg = random_hypergraph(seed, 40, 25, 1, 6, weighted=True)
    lv = _level(O, hg)
    pi = _pi(hg)
    z = np.random.default_rng(seed).standard_normal((lv.rows, 4))
    ref = pi @ z
    zj = z
    for _ in range(6):
        zj = O.sweep(lv, zj, 0.5, 0)
        np.testing.assert_allclose(pi @ zj, ref, rtol=1e-12, atol=1e-12)
    ze = O.sweep(lv, z, 0.5, 1)
    assert np.max(np.abs(pi @ ze - ref)) > 1e-6


@pytest.mark.parametrize("seed", SEEDS)
def test_maximum_principle(oracle_mod, seed):
    O = oracle_mod
    hg = random_hypergraph(seed, 40, 25, 1, 6, weighted=True)
    lv = _level(O, hg)
    z = np.random.default_rng(seed).standard_normal((lv.rows, 3))
    for _ in range(4):
        zn = O.sweep(lv, z, 0.7, 0)
        assert np.all(zn.max(axis=0) <= z.max(axis=0) + 1e-15)
        assert np.all(zn.min(axis=0) >= z.min(axis=0) - 1e-15)
        z = zn


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_limit_is_pi_weighted_component_mean(oracle_mod, seed):
    O = oracle_mod
    hg = random_hypergraph(seed, 30, 15, 2, 5, weighted=True)
    lv = _level(O, hg)
    comp = _components(hg)
    pi = _pi(hg)
    z0 = np.random.default_rng(seed).standard_normal((lv.rows, 2))
    z = z0
    for _ in range(3000):
        z = O.sweep(lv, z, 0.5, 0)
    for c in np.unique(comp):
        m = comp == c
        if pi[m].sum() == 0:     # isolated node: a fixed point
            np.testing.assert_allclose(z[m], z0[m], atol=1e-13)
            continue
        mean = (pi[m] @ z0[m]) / pi[m].sum()
        np.testing.assert_allclose(z[m], np.broadcast_to(mean, z[m].shape), atol=1e-9)


@pytest.mark.parametrize("seed", [0, 1])
def test_linearity_columns_identity_relabel(oracle_mod, seed):
    O = oracle_mod
    hg = random_hypergraph(seed, 30, 18, 1, 5, weighted=True)
    lv = _level(O, hg)
    rng = np.random.default_rng(seed)
    x, y = rng.standard_normal((2, lv.rows, 5))
    a, b = 1.7, -0.3
    for order in (0, 1):
        np.testing.assert_allclose(O.sweep(lv, a * x + b * y, 0.5, order),
                                   a * O.sweep(lv, x, 0.5, order) + b * O.sweep(lv, y, 0.5, order),
                                   atol=1e-13)
        full = O.sweep(lv, x, 0.5, order)
        for c in range(5):
            np.testing.assert_array_equal(O.sweep(lv, x[:, c:c + 1], 0.5, order)[:, 0], full[:, c])
        np.testing.assert_array_equal(O.sweep(lv, x, 0.0, order), x)
    # relabel nodes and hyperedges: the output is relabelled the same way
    pv = rng.permutation(hg.n_nodes)
    pe = rng.permutation(hg.n_edges)
    inv_v = np.argsort(pv)
    members = [sorted(int(inv_v[v]) for v in hg.edge_idx[hg.edge_ptr[e]:hg.edge_ptr[e + 1]]) for e in pe]
    ptr = np.concatenate([[0], np.cumsum([len(m) for m in members])]).astype(np.int64)
    idx = np.array([v for m in members for v in m], dtype=np.int32)
    w2 = hg.edge_w[pe]
    lv2 = O.Level(hg.n_nodes, hg.n_edges, ptr, idx, w2)
    perm_rows = np.concatenate([pv, hg.n_nodes + pe])      # new row r holds old row perm_rows[r]
    out2 = O.sweep(lv2, x[perm_rows], 0.5, 0)
    np.testing.assert_allclose(out2, O.sweep(lv, x, 0.5, 0)[perm_rows], atol=1e-13)


def test_refine_zero_sweeps_is_projection_chain(oracle_mod):
    O = oracle_mod
    hg = random_hypergraph(7, 60, 30, 2, 5, weighted=False)
    levels, maps = O.build_hierarchy(hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, None, 2)
    zc = np.random.default_rng(0).standard_normal((levels[2].rows, 3))
    out = O.refine(levels, maps, zc, [0, 0, 0], 0.5)
    P1 = projection_matrix(O.rowmap(levels[1], maps[1]), levels[2].rows)
    P0 = projection_matrix(O.rowmap(levels[0], maps[0]), levels[1].rows)
    np.testing.assert_array_equal(out, P0 @ P1 @ zc)


def test_refine_equals_dense_chain(oracle_mod):
    """Multi-level refinement as a product of dense matrices: per level, K
    sweep matrices after the projection (coarsest level first)."""
    O = oracle_mod
    hg = random_hypergraph(3, 45, 30, 1, 5, weighted=True)
    levels, maps = O.build_hierarchy(hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, hg.edge_w, 2)
    K = [3, 2, 4]
    zc = np.random.default_rng(1).standard_normal((levels[2].rows, 2))
    out, res = O.refine(levels, maps, zc, K, 0.5, return_residuals=True)
    z = zc
    ref_res = []
    for lvl in (2, 1, 0):
        lv = levels[lvl]
        if lvl < 2:
            z = projection_matrix(O.rowmap(lv, maps[lvl]), levels[lvl + 1].rows) @ z
        M = jacobi_matrix(star_adjacency(lv.n_nodes, lv.n_edges, lv.eptr, lv.eidx, lv.w), 0.5)
        for _ in range(K[lvl]):
            zn = M @ z
            ref_res.append(np.linalg.norm(zn - z))
            z = zn
    assert _rel(out, z) < 1e-13
    np.testing.assert_allclose(res, ref_res, rtol=1e-12)
