"""Pins for the oracle's reverse mode: the transpose of the dense sweep matrix,
the dot-product identity, and central finite differences in FP64 through
projection + several sweeps (for the coarse embedding and for the
per-hyperedge log-weights), plus the cross-entropy head."""
import numpy as np
import pytest

from hypothesis import given, settings
from hypothesis import strategies as st

from synth import random_hypergraph
from tests.dense_ref import edge_first_matrix, jacobi_matrix, star_adjacency


def _level(O, hg):
    return O.Level(hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, hg.edge_w)


@pytest.mark.parametrize("seed", range(4))
def test_vjp_is_dense_transpose_and_dot_identity(oracle_mod, seed):
    O = oracle_mod
    hg = random_hypergraph(seed, 33, 21, 1, 6, weighted=True)
    lv = _level(O, hg)
    rng = np.random.default_rng(seed)
    y = rng.standard_normal((lv.rows, 3))
    g = rng.standard_normal((lv.rows, 3))
    gy, _ = O.sweep_vjp(lv, y, g, 0.4)
    M = jacobi_matrix(star_adjacency(hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, hg.edge_w), 0.4)
    np.testing.assert_allclose(gy, M.T @ g, atol=1e-13)
    x = rng.standard_normal((lv.rows, 3))
    lhs = np.sum(O.sweep(lv, x, 0.4, 0) * g)
    rhs = np.sum(x * O.sweep_vjp(lv, x, g, 0.4)[0])
    assert abs(lhs - rhs) <= 1e-13 * max(1.0, abs(lhs))


@pytest.mark.parametrize("seed", range(4))
def test_edge_first_vjp_is_dense_transpose_and_dot_identity(oracle_mod, seed):
    """The edge-first sweep is the product of two partial relaxations (the
    hyperedge rows, then the node rows), so its reverse mode is that product's
    transpose.  The random hypergraphs include nodes in no hyperedge."""
    O = oracle_mod
    hg = random_hypergraph(40 + seed, 33, 21, 1, 6, weighted=True)
    lv = _level(O, hg)
    rng = np.random.default_rng(seed)
    y = rng.standard_normal((lv.rows, 3))
    g = rng.standard_normal((lv.rows, 3))
    gy, _ = O.sweep_vjp(lv, y, g, 0.7, order=1)
    A = star_adjacency(hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, hg.edge_w)
    M = edge_first_matrix(A, 0.7, hg.n_nodes)
    np.testing.assert_allclose(gy, M.T @ g, atol=1e-13)
    x = rng.standard_normal((lv.rows, 3))
    lhs = np.sum(O.sweep(lv, x, 0.7, 1) * g)
    rhs = np.sum(x * O.sweep_vjp(lv, x, g, 0.7, order=1)[0])
    assert abs(lhs - rhs) <= 1e-13 * max(1.0, abs(lhs))
    # the two orders differ, so neither reverse mode can stand in for the other
    assert np.abs(gy - O.sweep_vjp(lv, y, g, 0.7, order=0)[0]).max() > 1e-3


@pytest.mark.parametrize("seed", range(3))
def test_edge_first_weight_gradient_finite_differences(oracle_mod, seed):
    """dL/dw of one edge-first sweep, L = <sweep(y; w), G>, against central
    differences with steps exact in float32 (the weights' storage type)."""
    O = oracle_mod
    hg = random_hypergraph(60 + seed, 30, 18, 1, 6, weighted=True)
    lv = _level(O, hg)
    rng = np.random.default_rng(seed)
    y = rng.standard_normal((lv.rows, 4))
    G = rng.standard_normal((lv.rows, 4))
    w0 = np.asarray(hg.edge_w, dtype=np.float32)
    _, dw = O.sweep_vjp(lv, y, G, 0.6, w=w0, order=1)
    for e in range(hg.n_edges):
        step = np.float32(w0[e] * (1 + 1e-3)) - w0[e]
        wp = w0.copy(); wm = w0.copy()
        wp[e] += step; wm[e] -= step
        fd = (np.sum(O.sweep(lv, y, 0.6, 1, w=wp) * G) - np.sum(O.sweep(lv, y, 0.6, 1, w=wm) * G)) / (2 * float(step))
        assert abs(fd - dw[e]) <= 1e-6 * max(1.0, abs(dw[e])), (e, fd, dw[e])
    # scaling every weight by one factor leaves the sweep unchanged (node rows
    # take weighted means, hyperedge rows plain means): sum_e w_e dL/dw_e = 0
    assert abs(float(np.dot(w0.astype(np.float64), dw))) <= 1e-10 * max(1.0, np.abs(dw).sum())


@pytest.mark.parametrize("order", [0, 1])
@pytest.mark.parametrize("seed", range(3))
def test_finite_differences_theta_and_coarse(oracle_mod, seed, order):
    """L(theta, Zc) = <Z_k, G> with Z_k = k sweeps (weights exp(theta)) after
    projecting Zc, in either sweep order.  Central differences, h = 1e-6,
    FP64."""
    O = oracle_mod
    hg = random_hypergraph(20 + seed, 40, 25, 2, 6, weighted=False)
    fine = _level(O, hg)
    c = O.coarsen_level(fine)
    rng = np.random.default_rng(seed)
    theta = rng.uniform(-0.5, 0.5, size=hg.n_edges)
    zc = rng.standard_normal((c.coarse.rows, 3))
    G = rng.standard_normal((fine.rows, 3))
    k, omega = 4, 0.5

    def loss(th, zcoarse):
        zk, _, _ = O.finest_refine_vjp(fine, c, zcoarse, np.exp(th).astype(np.float32), k, omega, G, order)
        return float(np.sum(zk * G))

    # weights enter as float32, so dL/dw is checked with steps that are exact
    # in float32 (relative 1e-3); dL/dtheta = w dL/dw is the chain rule.
    w0 = np.exp(theta).astype(np.float32)
    _, gc, dw = O.finest_refine_vjp(fine, c, zc, w0, k, omega, G, order)
    h = 1e-6
    for e in range(0, hg.n_edges, 3):
        wp = w0.astype(np.float64).copy(); wm = wp.copy()
        step = np.float32(w0[e] * (1 + 1e-3)) - w0[e]          # exact float32 step
        wp[e] += step; wm[e] -= step
        lp = float(np.sum(O.finest_refine_vjp(fine, c, zc, wp.astype(np.float32), k, omega, G, order)[0] * G))
        lm = float(np.sum(O.finest_refine_vjp(fine, c, zc, wm.astype(np.float32), k, omega, G, order)[0] * G))
        fd = (lp - lm) / (2 * float(step))
        assert abs(fd - dw[e]) <= 1e-5 * max(1.0, abs(dw[e])), (e, fd, dw[e])
    for r in range(0, c.coarse.rows, 4):
        for col in range(3):
            zp = zc.copy(); zm = zc.copy()
            zp[r, col] += h; zm[r, col] -= h
            fd = (loss(theta, zp) - loss(theta, zm)) / (2 * h)
            assert abs(fd - gc[r, col]) <= 1e-6 * max(1.0, abs(gc[r, col]))


def test_ce_head_gradient(oracle_mod):
    O = oracle_mod
    rng = np.random.default_rng(0)
    z = rng.standard_normal((20, 8))
    W = rng.standard_normal((5, 8)) / 3
    b = rng.standard_normal(5)
    y = rng.integers(0, 5, size=20)
    loss, dz = O.ce_head(z, y, W, b)
    # closed form at W = 0: every class equally likely, loss = log C
    assert abs(O.ce_head(z, y, np.zeros_like(W), np.zeros_like(b))[0] - np.log(5)) < 1e-14
    h = 1e-6
    for i in range(0, 20, 3):
        for j in range(8):
            zp = z.copy(); zm = z.copy()
            zp[i, j] += h; zm[i, j] -= h
            fd = (O.ce_head(zp, y, W, b)[0] - O.ce_head(zm, y, W, b)[0]) / (2 * h)
            assert abs(fd - dz[i, j]) < 1e-8


@st.composite
def _tiny(draw):
    n = draw(st.integers(1, 9))
    m = draw(st.integers(0, 7))
    edges = [sorted(draw(st.sets(st.integers(0, n - 1), min_size=1, max_size=min(4, n)))) for _ in range(m)]
    w = [float(draw(st.sampled_from([0.5, 1.0, 2.0, 3.0]))) for _ in range(m)]
    omega = draw(st.sampled_from([0.25, 0.5, 1.0]))
    order = draw(st.sampled_from([0, 1]))
    seed = draw(st.integers(0, 2**31 - 1))
    return n, edges, w, omega, order, seed


@settings(max_examples=200, deadline=None)
@given(t=_tiny())
def test_vjp_properties_on_tiny_hypergraphs(t):
    """Either order on random tiny hypergraphs (empty hyperedge sets,
    isolated nodes, single-member hyperedges): dL/dy is the dense sweep
    matrix's transpose times g, and dL/dw equals central differences of the
    dense FP64 forward form, which shares no code with the oracle."""
    from oracle import oracle as O
    n, edges, w, omega, order, seed = t
    ptr = np.concatenate([[0], np.cumsum([len(e) for e in edges])]).astype(np.int64)
    idx = np.array([v for e in edges for v in e], dtype=np.int32)
    wf = np.array(w, dtype=np.float32)
    lv = O.Level(n, len(edges), ptr, idx, wf)
    rng = np.random.default_rng(seed)
    y = rng.standard_normal((lv.rows, 2))
    g = rng.standard_normal((lv.rows, 2))

    def dense(wv):
        A = star_adjacency(n, len(edges), ptr, idx, wv)
        return edge_first_matrix(A, omega, n) if order else jacobi_matrix(A, omega)

    gy, dw = O.sweep_vjp(lv, y, g, omega, wf, order)
    np.testing.assert_allclose(gy, dense(wf.astype(np.float64)).T @ g, atol=1e-12)
    h = 1e-6
    for e in range(len(edges)):
        wp = wf.astype(np.float64).copy(); wm = wp.copy()
        wp[e] += h; wm[e] -= h
        fd = (np.sum((dense(wp) @ y) * g) - np.sum((dense(wm) @ y) * g)) / (2 * h)
        assert abs(fd - dw[e]) <= 1e-6 * max(1.0, abs(fd)), (e, fd, dw[e])
