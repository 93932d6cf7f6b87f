"""The oracle against the hand-worked example in tests/golden/worked_example.txt
(Algorithm 2 sweeps in both orders, their reverse mode, Algorithm 1 coarsening,
the projection rule)."""
import numpy as np

from tests.golden_io import as_floats, read_fixture

FX = read_fixture("worked_example.txt")


def _level(O, weights=None):
    edges = [[int(v) for v in row] for row in FX["edge"]]
    ptr = np.concatenate([[0], np.cumsum([len(e) for e in edges])]).astype(np.int64)
    idx = np.array([v for e in edges for v in e], dtype=np.int32)
    n = int(FX["n_nodes"][0][0])
    return O.Level(n, len(edges), ptr, idx, weights)


def _col(key):
    return np.array(as_floats(FX[key][0]))[:, None]


def test_sweeps(oracle_mod):
    O = oracle_mod
    lv = _level(O)
    om = float(FX["omega"][0][0])
    z0 = _col("z0")
    z1 = O.sweep(lv, z0, om, 0)
    z2 = O.sweep(lv, z1, om, 0)
    np.testing.assert_allclose(z1, _col("jacobi1"), rtol=0, atol=1e-15)
    np.testing.assert_allclose(z2, _col("jacobi2"), rtol=0, atol=1e-15)
    pi = _col("pi")[:, 0]
    for z in (z0, z1, z2):
        assert abs(pi @ z[:, 0] - float(FX["conserved"][0][0])) < 1e-13
    np.testing.assert_allclose(O.sweep(lv, z0, om, 1), _col("edgefirst1"), atol=1e-15)
    lvw = _level(O, np.array(as_floats(FX["weights"][0]), dtype=np.float32))
    np.testing.assert_allclose(O.sweep(lvw, z0, om, 0), _col("jacobi1_weighted"), atol=1e-15)


def test_vjp(oracle_mod):
    O = oracle_mod
    lv = _level(O)
    z0 = _col("z0")
    g = np.zeros_like(z0)
    g[int(FX["vjp_target_row"][0][0]), 0] = 1.0
    gy, dw = O.sweep_vjp(lv, z0, g, float(FX["omega"][0][0]))
    np.testing.assert_allclose(gy, _col("vjp_gz0"), atol=1e-15)
    np.testing.assert_allclose(dw, as_floats(FX["vjp_dw"][0]), atol=1e-15)


def test_vjp_edge_first(oracle_mod):
    O = oracle_mod
    lv = _level(O)
    y = _col("ef_vjp_y")
    g = np.zeros_like(y)
    g[int(FX["vjp_target_row"][0][0]), 0] = 1.0
    gy, dw = O.sweep_vjp(lv, y, g, float(FX["omega"][0][0]), order=1)
    np.testing.assert_allclose(gy, _col("ef_vjp_gz0"), atol=1e-15)
    np.testing.assert_allclose(dw, as_floats(FX["ef_vjp_dw"][0]), atol=1e-15)


def test_coarsen_and_project(oracle_mod):
    O = oracle_mod
    lv = _level(O)
    c = O.coarsen_level(lv)
    assert list(c.node_rep) == [int(v) for v in FX["node_rep"][0]]
    assert list(c.edge_rep) == [int(v) for v in FX["edge_rep"][0]]
    assert c.coarse.n_nodes == int(FX["coarse_nodes"][0][0])
    assert [list(c.coarse.eidx[c.coarse.eptr[e]:c.coarse.eptr[e + 1]]) for e in range(c.coarse.n_edges)] == \
        [[int(v) for v in row] for row in FX["coarse_edge"]]
    rm = O.rowmap(lv, c)
    assert list(rm) == [int(v) for v in FX["rowmap"][0]]
    np.testing.assert_array_equal(O.project(rm, _col("zc")), _col("projected"))
