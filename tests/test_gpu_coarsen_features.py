"""GPU coarsening with node features (Section 3.1, Algorithm 1 with X)
against the oracle: maps, coarse levels and the coarse feature matrices must
be equal bit for bit (integer work; the cosine decision is one FP64 product
and one FP64 quotient of exact integers on both sides)."""
import numpy as np
import pytest

from tests.cases import CONFIGS, make_hypergraph, random_hypergraph

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2103_09660_amd as H
    return H


def _compare(O, H, hg, x, n_coarsen, what):
    import torch
    levels, maps, feats = O.build_hierarchy_features(hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, hg.edge_w,
                                                     x, n_coarsen)
    lv0 = H.DeviceLevel.from_host(H.HostLevel(hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, hg.edge_w), "cuda")
    dl, dm, df = H.coarsen_hierarchy_features_device(lv0, torch.as_tensor(x).cuda(), n_coarsen)
    for l in range(n_coarsen):
        nrep, erep = (t.cpu().numpy() for t in dm[l])
        assert np.array_equal(nrep, maps[l].node_rep), f"{what}: node_rep of step {l}"
        assert np.array_equal(erep, maps[l].edge_rep), f"{what}: edge_rep of step {l}"
        got, ref = dl[l + 1].to_host(), levels[l + 1]
        assert (got.n_nodes, got.n_edges, got.nnz) == (ref.n_nodes, ref.n_edges, ref.nnz), f"{what}: sizes {l}"
        assert np.array_equal(got.edge_ptr, ref.eptr) and np.array_equal(got.edge_idx, ref.eidx), f"{what}: {l}"
        assert np.array_equal(df[l + 1].cpu().numpy(), feats[l + 1]), f"{what}: coarse features of step {l}"


@pytest.mark.parametrize("seed,n_nodes,n_edges,hi,k,weights", [
    (0, 1, 1, 1, 4, "none"), (1, 10, 6, 3, 4, "int"), (2, 80, 50, 6, 12, "none"), (3, 500, 300, 8, 64, "float"),
    (4, 2000, 1500, 12, 128, "int"), (5, 3000, 1000, 40, 500, "none"), (6, 700, 900, 5, 1000, "int"),
    (7, 20000, 12000, 20, 256, "none")])
def test_random_hypergraphs(oracle_mod, H, seed, n_nodes, n_edges, hi, k, weights):
    """Empty documents and repeated documents give exact cosine ties that the
    featureless order must break the same way on both sides."""
    from synth import bag_of_words
    hg = random_hypergraph(seed, n_nodes, n_edges, 1, hi, weighted=weights != "none",
                           integer_weights=weights == "int")
    x = bag_of_words(500 + seed, n_nodes, k, 1, min(30, k), empty_frac=0.05, repeat_frac=0.2)
    _compare(oracle_mod, H, hg, x, 3, f"seed {seed}")


@pytest.mark.parametrize("name", ["bow-20k", "bow-1m"])
def test_named_workload_hierarchy(oracle_mod, H, name):
    from synth import node_features
    cfg = CONFIGS[name]
    _compare(oracle_mod, H, make_hypergraph(cfg), node_features(cfg), cfg.levels, name)


def test_zero_features_match_featureless(H):
    import torch
    hg = random_hypergraph(21, 5000, 4000, 1, 9, weighted=True, integer_weights=True)
    lv = H.DeviceLevel.from_host(H.HostLevel(hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, hg.edge_w))
    a = H.coarsen_level_device(lv)
    b = H.coarsen_level_features_device(lv, torch.zeros((hg.n_nodes, 16), dtype=torch.int32, device="cuda"))
    for u, v in zip(a[:2], b[:2]):
        assert torch.equal(u, v)
    assert torch.equal(a[2].edge_idx, b[2].edge_idx) and int(b[3].abs().sum()) == 0


def test_dirty_workspace_and_reuse(oracle_mod, H):
    import torch
    from synth import bag_of_words
    O = oracle_mod
    big = random_hypergraph(31, 4000, 3000, 1, 9)
    small = random_hypergraph(32, 900, 500, 1, 6, weighted=False)
    k = 64
    ws = torch.full((H.coarsen_features_workspace_bytes(big.n_nodes, big.n_edges, big.nnz, k),), 255,
                    dtype=torch.uint8, device="cuda")
    for i, hg in enumerate((big, small, big)):
        x = bag_of_words(40 + i, hg.n_nodes, k, 2, 10, repeat_frac=0.3)
        c, xc = O.coarsen_level_features(O.Level(hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, hg.edge_w), x)
        lv = H.DeviceLevel.from_host(H.HostLevel(hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, hg.edge_w))
        nrep, erep, coarse, xg = H.coarsen_level_features_device(lv, torch.as_tensor(x).cuda(), ws)
        assert np.array_equal(nrep.cpu().numpy(), c.node_rep) and np.array_equal(erep.cpu().numpy(), c.edge_rep)
        assert np.array_equal(xg.cpu().numpy(), xc)


def test_invalid_features_are_rejected(H):
    import ctypes
    import torch
    from paper_2103_09660_amd import _lib as L
    hg = random_hypergraph(5, 100, 60, 1, 5)
    lv = H.DeviceLevel.from_host(H.HostLevel(hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, hg.edge_w))
    x = torch.ones((hg.n_nodes, 8), dtype=torch.int32, device="cuda")
    x[3, 5] = -1
    with pytest.raises(H.HnvError) as ei:
        H.coarsen_level_features_device(lv, x)
    assert ei.value.status == L.HNV_EINVAL
    x = torch.zeros((hg.n_nodes, 8), dtype=torch.int32, device="cuda")
    x[0, 0] = 2 ** 31 - 1
    x[1, 1] = 1                                   # total reaches 2^31
    with pytest.raises(H.HnvError) as ei:
        H.coarsen_level_features_device(lv, x)
    assert ei.value.status == L.HNV_EINVAL
    x[1, 1] = 0                                   # total 2^31 - 1 is allowed
    H.coarsen_level_features_device(lv, x)
    # k not a multiple of 4, and k = 0, through the C ABI
    need = H.coarsen_features_workspace_bytes(hg.n_nodes, hg.n_edges, hg.nnz, 8)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    out = [torch.empty(max(n, 1), dtype=dt, device="cuda") for n, dt in
           ((hg.n_nodes, torch.int32), (hg.n_edges, torch.int32), (hg.n_edges + 1, torch.int32),
            (hg.nnz, torch.int32), (hg.n_edges, torch.float32))]
    cx = torch.empty((hg.n_nodes, 8), dtype=torch.int32, device="cuda")
    sizes = (ctypes.c_int64 * 3)()
    for k in (6, 0):
        st = L.lib().hnv_coarsen_level_features_device(
            hg.n_nodes, hg.n_edges, hg.nnz, lv.edge_ptr.data_ptr(), lv.edge_idx.data_ptr(), lv.edge_w.data_ptr(),
            x.data_ptr(), k, *[t.data_ptr() for t in out[:4]], out[4].data_ptr(), cx.data_ptr(),
            ctypes.cast(sizes, L.i64p), ws.data_ptr(), need, None)
        assert st == L.HNV_EUNSUPPORTED


def test_features_without_hyperedges(H):
    """Nodes only: every node is its own coarse node and X' = X; and an empty
    level."""
    import torch
    x = torch.randint(0, 4, (9, 12), dtype=torch.int32, device="cuda")
    lv = H.DeviceLevel(9, 0, 0, torch.zeros(1, dtype=torch.int32, device="cuda"),
                       torch.zeros(0, dtype=torch.int32, device="cuda"))
    nrep, erep, c, xc = H.coarsen_level_features_device(lv, x)
    assert nrep.cpu().tolist() == list(range(9)) and (c.n_nodes, c.n_edges, c.nnz) == (9, 0, 0)
    assert torch.equal(xc, x)
    lv = H.DeviceLevel(0, 0, 0, torch.zeros(1, dtype=torch.int32, device="cuda"),
                       torch.zeros(0, dtype=torch.int32, device="cuda"))
    nrep, erep, c, xc = H.coarsen_level_features_device(lv, torch.zeros((0, 8), dtype=torch.int32, device="cuda"))
    assert (c.n_nodes, c.n_edges, c.nnz) == (0, 0, 0) and xc.shape[0] == 0
