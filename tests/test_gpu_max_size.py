"""The index range at its limit: a level with 2.0e9 incidences (the C ABI
takes up to 2^31 - 1), built into a plan on the GPU, one forward sweep
with its residual and one reverse sweep with the split weight gradient.
The hypergraph is a band (hyperedge e holds nodes e .. e+K-1), so every
window of it is a small hypergraph of its own: the oracle sweeps windows
at the start, the middle and the end of the index range, and the rows
whose neighbourhoods lie inside a window must match it.  The residual
is checked against its definition, ||Z' - Z||_F, taken in FP64."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

K = 100                     # members per hyperedge (above the lane-group bound: wavefront tier)
E = 20_000_000              # hyperedges: nnz = 2.0e9
N = E + K - 1               # nodes
D = 8
OMEGA = 0.5
W = 4 * K                   # window width in nodes


def _z0(rows, torch):
    """A deterministic embedding, the same on the host and the device."""
    r = rows.to(torch.float64)[:, None]
    c = torch.arange(D, dtype=torch.float64, device=rows.device)[None, :]
    return torch.sin(r * 1e-3 + c * 0.7).to(torch.float32)


def _window(O, a):
    """Nodes [a, a+W) and the hyperedges inside them, renumbered from 0."""
    e0, e1 = a, a + W - K + 1
    ptr = np.arange(e1 - e0 + 1, dtype=np.int64) * K
    idx = (np.arange(e1 - e0)[:, None] + np.arange(K)[None, :]).astype(np.int32).ravel()
    return O.Level(W, e1 - e0, ptr, idx, None), e0, e1


def test_index_range_limit(oracle_mod):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2103_09660_amd as H
    O = oracle_mod
    nnz = E * K
    assert nnz < 2 ** 31 - 1 and N + E < 2 ** 31 - 1
    print(f"band hypergraph: {N} nodes, {E} hyperedges, {nnz} incidences", flush=True)
    dev = torch.device("cuda")
    ptr = torch.arange(E + 1, dtype=torch.int32, device=dev) * K
    idx = (torch.arange(E, dtype=torch.int32, device=dev)[:, None] +
           torch.arange(K, dtype=torch.int32, device=dev)[None, :]).reshape(-1)
    lv = H.DeviceLevel(N, E, nnz, ptr, idx)
    print("plan", flush=True)
    plan = H.Plan.from_device([lv], [], D, "f32", options={"chunk": 64})
    del ptr, idx, lv
    rows = N + E
    z0 = _z0(torch.arange(rows, device=dev), torch)
    resid = torch.zeros(1, dtype=torch.float64, device=dev)
    print("forward sweep", flush=True)
    z1 = plan.sweep(0, z0, OMEGA, resid=resid)
    ref_resid = torch.linalg.vector_norm((z1.double() - z0.double()).reshape(-1)).item()
    assert abs(resid.item() - ref_resid) <= 1e-6 * ref_resid
    print("reverse sweep", flush=True)
    g = _z0(torch.arange(rows, device=dev) * 7 + 3, torch)
    dw = torch.zeros(E, dtype=torch.float32, device=dev)
    nacc = torch.zeros(N, dtype=torch.float32, device=dev)
    g1 = plan.sweep_adjoint(0, g, z0, z1, OMEGA, dw=dw, node_acc=nacc)
    plan.weight_grad_finish(0, nacc, dw)
    torch.cuda.synchronize()
    for a in (0, N // 2, N - W):
        print(f"window at node {a}", flush=True)
        lw, e0, e1 = _window(O, a)
        grow = torch.cat([torch.arange(a, a + W), N + torch.arange(e0, e1)]).to(dev)   # window rows, global ids
        y = z0[grow].cpu().numpy()
        gl = g[grow].cpu().numpy()
        ref = O.sweep(lw, y, OMEGA)
        ref_g, ref_dw = O.sweep_vjp(lw, y, gl, OMEGA)
        got = z1[grow].cpu().numpy()
        got_g = g1[grow].cpu().numpy()
        # window nodes whose K hyperedges all lie in the window (at the ends of
        # the band a node has fewer, and the window holds all of them) ...
        node_lo = 0 if a == 0 else K - 1
        node_hi = W - 1 if a + W - K >= E - 1 else W - K
        node_rows = np.arange(node_lo, node_hi + 1)
        # ... every window hyperedge sees all its members; in reverse mode a
        # hyperedge also needs each member's weight sum and neighbour mean
        edge_rows = np.arange(e1 - e0)
        inner_edges = np.arange(node_lo, min(node_hi - K + 2, e1 - e0))
        for what, gv, rv, rr in (("forward node rows", got, ref, node_rows),
                                 ("forward hyperedge rows", got, ref, W + edge_rows),
                                 ("reverse node rows", got_g, ref_g, node_rows),
                                 ("reverse hyperedge rows", got_g, ref_g, W + inner_edges)):
            err = np.max(np.abs(gv[rr] - rv[rr])) / np.max(np.abs(rv[rr]))
            assert err <= 1e-5, f"{what} at node {a}: {err:.3e}"
        got_dw = dw[e0:e1].cpu().numpy()[inner_edges]
        err = np.max(np.abs(got_dw - ref_dw[inner_edges])) / np.max(np.abs(ref_dw[inner_edges]))
        assert err <= 1e-4, f"weight gradient at node {a}: {err:.3e}"
