"""The GPU library against the hand-worked example in
tests/golden/worked_example.txt directly, not through the oracle: sweeps in
both orders (unit and non-unit weights), the reverse sweep and its weight
gradient in both orders, coarsening on the host and on the GPU, and the
projection.  The example has d = 1; the plans run d = 8 with column c
holding (c + 1) times the example (every operation is linear in Z), and the
cotangents live in column 0 only, so the weight gradients are the
example's own."""
import numpy as np
import pytest

from tests.golden_io import as_floats, read_fixture

pytestmark = pytest.mark.gpu

FX = read_fixture("worked_example.txt")
D = 8
SCALE = np.arange(1, D + 1, dtype=np.float64)


@pytest.fixture(scope="module")
def H():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2103_09660_amd as H
    return H


def _host_level(H, weights=None):
    edges = [[int(v) for v in row] for row in FX["edge"]]
    ptr = np.concatenate([[0], np.cumsum([len(e) for e in edges])]).astype(np.int64)
    idx = np.array([v for e in edges for v in e], dtype=np.int32)
    w = None if weights is None else np.asarray(weights, dtype=np.float32)
    return H.HostLevel(int(FX["n_nodes"][0][0]), len(edges), ptr, idx, w)


def _vals(key):
    return np.array(as_floats(FX[key][0]))


def _wide(col):
    """[rows x D] FP32 device matrix with column c = (c + 1) * col."""
    import torch
    return torch.as_tensor((col[:, None] * SCALE[None, :]).astype(np.float32)).cuda()


def _check_wide(got, col, what):
    ref = col[:, None] * SCALE[None, :]
    np.testing.assert_allclose(got.cpu().numpy().astype(np.float64), ref, rtol=1e-6, atol=1e-6, err_msg=what)


def _plan(H, order, weights=None):
    return H.Plan(H.Hierarchy([_host_level(H, weights)], []), D, "f32", options={"order": order})


def test_sweeps(H):
    om = float(FX["omega"][0][0])
    z0 = _vals("z0")
    jac = _plan(H, "jacobi")
    z1 = jac.sweep(0, _wide(z0), om)
    _check_wide(z1, _vals("jacobi1"), "Jacobi sweep 1")
    _check_wide(jac.sweep(0, z1, om), _vals("jacobi2"), "Jacobi sweep 2")
    weighted = _plan(H, "jacobi", as_floats(FX["weights"][0]))
    _check_wide(weighted.sweep(0, _wide(z0), om), _vals("jacobi1_weighted"), "weighted Jacobi sweep")
    ef = _plan(H, "edge_first")
    _check_wide(ef.sweep(0, _wide(z0), om), _vals("edgefirst1"), "edge-first sweep")
    zi = _wide(z0)
    ef.sweep(0, zi, om, out=zi)
    _check_wide(zi, _vals("edgefirst1"), "edge-first sweep in place")


@pytest.mark.parametrize("order,y_key,g_key,dw_key", [("jacobi", "z0", "vjp_gz0", "vjp_dw"),
                                                      ("edge_first", "ef_vjp_y", "ef_vjp_gz0", "ef_vjp_dw")])
def test_reverse_sweep(H, order, y_key, g_key, dw_key):
    import torch
    om = float(FX["omega"][0][0])
    plan = _plan(H, order)
    y = _wide(_vals(y_key))
    z = plan.sweep(0, y, om)
    g = torch.zeros_like(y)
    g[int(FX["vjp_target_row"][0][0]), 0] = 1.0
    n_edges = len(FX["edge"])
    for split in (False, True):
        dw = torch.zeros(n_edges, dtype=torch.float32, device="cuda")
        nacc = torch.zeros(int(FX["n_nodes"][0][0]), dtype=torch.float32, device="cuda") if split else None
        gy = plan.sweep_adjoint(0, g, y, z, om, dw=dw, node_acc=nacc)
        if split:
            plan.weight_grad_finish(0, nacc, dw)
        want = np.zeros((len(_vals(g_key)), D))
        want[:, 0] = _vals(g_key)
        np.testing.assert_allclose(gy.cpu().numpy(), want, rtol=1e-6, atol=1e-7, err_msg=f"{order} dL/dy")
        np.testing.assert_allclose(dw.cpu().numpy(), _vals(dw_key), rtol=1e-6, atol=1e-7,
                                   err_msg=f"{order} dL/dw (split={split})")


def test_coarsen_and_project(H):
    fine = _host_level(H)
    m, c = H.coarsen_level(fine)
    assert list(m.node_rep[:fine.n_nodes]) == [int(v) for v in FX["node_rep"][0]]
    assert list(m.edge_rep[:fine.n_edges]) == [int(v) for v in FX["edge_rep"][0]]
    assert c.n_nodes == int(FX["coarse_nodes"][0][0])
    assert [list(c.edge_idx[c.edge_ptr[e]:c.edge_ptr[e + 1]]) for e in range(c.n_edges)] == \
        [[int(v) for v in row] for row in FX["coarse_edge"]]
    nrep, erep, cd = H.coarsen_level_device(H.DeviceLevel.from_host(fine, "cuda"))
    assert list(nrep.cpu().numpy()) == [int(v) for v in FX["node_rep"][0]]
    assert list(erep.cpu().numpy()) == [int(v) for v in FX["edge_rep"][0]]
    plan = H.Plan(H.Hierarchy([fine, c], [m]), D, "f32")
    _check_wide(plan.project(0, _wide(_vals("zc"))), _vals("projected"), "projection")
