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

from tests.cases import assert_close

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _release_device_memory():
    """These tests take up to about 150 GB of device memory: start and end
    with torch's cached blocks returned."""
    import torch
    if torch.cuda.is_available():
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    yield
    if torch.cuda.is_available():
        import gc
        gc.collect()
        torch.cuda.synchronize()
        torch.cuda.empty_cache()

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
            assert_close(gv[rr], rv[rr], 1e-5, f"{what} at node {a}")
        got_dw = dw[e0:e1].cpu().numpy()[inner_edges]
        assert_close(got_dw, ref_dw[inner_edges], 1e-4, f"weight gradient at node {a}")
    # hyperedge-prediction features over the same 2.0e9 memberships: every
    # hyperedge as a candidate set, scored on the node rows of Z'
    del plan, g, g1, dw, nacc
    torch.cuda.empty_cache()
    print("candidate scores", flush=True)
    cptr = torch.arange(E + 1, dtype=torch.int32, device=dev) * K
    cidx = (torch.arange(E, dtype=torch.int32, device=dev)[:, None] +
            torch.arange(K, dtype=torch.int32, device=dev)[None, :]).reshape(-1)
    sp = H.ScorePlan.from_device(cptr, cidx, N, D, "f32")
    del cptr, cidx
    zn = z1[:N].contiguous()
    var = sp.score(zn, "variance")
    torch.cuda.synchronize()
    for c0 in (0, E // 2, E - 3):
        cs = np.arange(c0, c0 + 3)
        nodes = np.arange(c0, c0 + 3 + K - 1)
        zsub = zn[torch.as_tensor(nodes, device=dev)].cpu().numpy()
        lptr = np.arange(4, dtype=np.int64) * K
        lidx = (np.arange(3)[:, None] + np.arange(K)[None, :]).astype(np.int32).ravel()
        ref = O.score_candidates(zsub, lptr, lidx, "variance")
        got = var[torch.as_tensor(cs, device=dev)].cpu().numpy()
        assert_close(got, ref, 1e-5, f"scores of candidates {c0}..")


def test_index_range_limit_two_levels(oracle_mod):
    """The same scale through the GPU coarsening, the fused projection sweep
    and the projection adjoint.  Level 0 adds to the band a partition of
    the nodes into blocks of B, one heavier hyperedge per block (ids first),
    so that by the featureless rule every node joins its block's hyperedge:
    the coarse level has one node per block, the block hyperedges are
    removed and each band hyperedge keeps the one or two blocks it touches.
    That coarse level is small enough for the oracle; the GPU coarsening
    must produce it exactly, and the refinement of both levels must match
    the oracle on windows of level 0."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2103_09660_amd as H
    O = oracle_mod
    B, M = 100, 198_000
    n = B * M
    eb = n - K + 1                         # band hyperedges
    nnz = M * B + eb * K
    assert nnz < 2 ** 31 - 1
    print(f"two levels: {n} nodes, {M} block + {eb} band hyperedges, {nnz} incidences", flush=True)
    dev = torch.device("cuda")
    i32 = dict(dtype=torch.int32, device=dev)
    ptr = torch.cat([torch.arange(M, **i32) * B, M * B + torch.arange(eb + 1, **i32) * K])
    idx = torch.cat([torch.arange(n, **i32),
                     (torch.arange(eb, **i32)[:, None] + torch.arange(K, **i32)[None, :]).reshape(-1)])
    w = torch.cat([torch.full((M,), 2.0, device=dev), torch.ones(eb, device=dev)])
    lv0 = H.DeviceLevel(n, M + eb, nnz, ptr, idx, w)
    print("coarsening", flush=True)
    nrep, erep, lv1 = H.coarsen_level_device(lv0)
    # the coarse level by the featureless rule, written out
    assert torch.equal(nrep, torch.arange(n, **i32) // B)
    assert torch.equal(erep, torch.cat([torch.full((M,), -1, **i32), torch.arange(eb, **i32)]))
    first = torch.arange(eb, **i32) // B
    last = (torch.arange(eb, **i32) + K - 1) // B
    two = last != first
    sizes = 1 + two.to(torch.int32)
    assert (lv1.n_nodes, lv1.n_edges, lv1.nnz) == (M, eb, int(sizes.sum().item()))
    assert torch.equal(lv1.edge_ptr, torch.cat([torch.zeros(1, **i32), torch.cumsum(sizes, 0).to(torch.int32)]))
    members = torch.stack([first, torch.where(two, last, first)], 1).reshape(-1)
    keep = torch.stack([torch.ones_like(two), two], 1).reshape(-1)
    assert torch.equal(lv1.edge_idx, members[keep])
    assert torch.equal(lv1.edge_w, torch.ones(eb, device=dev))
    print("plan", flush=True)
    plan = H.Plan.from_device([lv0, lv1], [(nrep, erep)], D, "f32", options={"chunk": 64})
    rows1 = M + eb
    zc = _z0(torch.arange(rows1, device=dev) * 3 + 1, torch)
    out, _, _ = plan.refine(zc, [1, 1], OMEGA)
    print("projection adjoint", flush=True)
    gf = _z0(torch.arange(n + M + eb, device=dev) * 5 + 2, torch)
    gc = plan.project_adjoint(0, gf)
    rowmap = torch.cat([torch.arange(n, device=dev) // B,            # node v -> its block
                        torch.arange(M, device=dev),                  # a removed block hyperedge -> its block
                        M + torch.arange(eb, device=dev)])            # a band hyperedge -> its coarse row
    ref_gc = torch.zeros(rows1, D, dtype=torch.float64, device=dev).index_add_(0, rowmap, gf.double())
    # per element: |got - ref| <= 1e-5 (|ref| + rms(ref)), on the device
    rms = float(ref_gc.pow(2).mean().sqrt())
    assert bool(((gc.double() - ref_gc).abs() <= 1e-5 * (ref_gc.abs() + rms)).all())
    torch.cuda.synchronize()
    # the oracle: the coarse level as written out above, one sweep there, then windows of level 0
    print("oracle, coarse level", flush=True)
    f, l, t = first.cpu().numpy(), last.cpu().numpy(), two.cpu().numpy()
    c_ptr = np.concatenate([[0], np.cumsum(1 + t)]).astype(np.int64)
    c_idx = np.stack([f, np.where(t, l, f)], 1).reshape(-1)[np.stack([np.ones_like(t), t], 1).reshape(-1)]
    z1 = O.sweep(O.Level(M, eb, c_ptr, c_idx.astype(np.int32), np.ones(eb, np.float32)),
                 zc.cpu().numpy(), OMEGA)
    outn = out.cpu().numpy()
    Wb = 4                                   # window: 4 blocks of nodes
    for blk in (0, M // 2, M - Wb):
        a, wn = blk * B, Wb * B
        print(f"window at node {a}", flush=True)
        e0, e1 = a, min(a + wn - K + 1, eb)  # band hyperedges inside the window
        blocks = np.arange(blk, blk + Wb)
        h_ptr = np.arange(Wb + 1, dtype=np.int64) * B
        b_ptr = Wb * B + np.arange(e1 - e0 + 1, dtype=np.int64) * K
        lw_idx = np.concatenate([np.arange(wn), (np.arange(e1 - e0)[:, None] + np.arange(K)[None, :]).ravel()])
        lw = O.Level(wn, Wb + e1 - e0, np.concatenate([h_ptr, b_ptr[1:]]), lw_idx.astype(np.int32),
                     np.concatenate([np.full(Wb, 2.0), np.ones(e1 - e0)]).astype(np.float32))
        # start values: level 0 rows projected from the swept coarse level
        start = np.concatenate([z1[(a + np.arange(wn)) // B], z1[blocks], z1[M + np.arange(e0, e1)]])
        ref = O.sweep(lw, start, OMEGA)
        grow = np.concatenate([a + np.arange(wn), n + blocks, n + M + np.arange(e0, e1)])
        got = outn[grow]
        node_lo = 0 if a == 0 else K - 1
        node_hi = wn - 1 if a + wn - K >= eb - 1 else wn - K
        rr = np.concatenate([np.arange(node_lo, node_hi + 1), wn + np.arange(Wb + e1 - e0)])
        assert_close(got[rr], ref[rr], 1e-5, f"window at node {a}")


def test_cast_beyond_one_grid_dimension():
    """A conversion of 2^32 + 5 elements (a launch folded into three grid
    rows) rounds every element to nearest even, as torch does."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2103_09660_amd as H
    n = 2 ** 32 + 5
    x = torch.empty(n, dtype=torch.float32, device="cuda")
    x.uniform_(-3.0, 3.0)
    y = H.cast(x, "bf16")
    assert torch.equal(y, x.to(torch.bfloat16))
    del y
    back = H.cast(x[-1000:].to(torch.bfloat16).contiguous(), "f32")
    assert torch.equal(back, x[-1000:].to(torch.bfloat16).float())
