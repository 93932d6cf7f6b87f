"""GPU coarsening (Section 3.1, Algorithm 1, featureless) against the oracle:
node and hyperedge maps and every coarse level must be equal bit for bit
(integer work; weights are copied, never computed)."""
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


def _compare(O, H, n_nodes, n_edges, eptr, eidx, w, n_coarsen, what):
    levels, maps = O.build_hierarchy(n_nodes, n_edges, eptr, eidx, w, n_coarsen)
    dl, dm = H.coarsen_hierarchy_device(
        H.DeviceLevel.from_host(H.HostLevel(n_nodes, n_edges, eptr, eidx, w), "cuda"), n_coarsen)
    for l in range(n_coarsen):
        nrep, erep = (t.cpu().numpy() for t in dm[l])
        assert np.array_equal(nrep, maps[l].node_rep), f"{what}: node_rep of step {l}"
        assert np.array_equal(erep, maps[l].edge_rep), f"{what}: edge_rep of step {l}"
        got, ref = dl[l + 1].to_host(), levels[l + 1]
        assert (got.n_nodes, got.n_edges, got.nnz) == (ref.n_nodes, ref.n_edges, ref.nnz), f"{what}: sizes {l}"
        assert np.array_equal(got.edge_ptr, ref.eptr), f"{what}: coarse offsets of step {l}"
        assert np.array_equal(got.edge_idx, ref.eidx), f"{what}: coarse members of step {l}"
        if ref.w is None:
            assert got.edge_w is None
        else:
            assert np.array_equal(got.edge_w.view(np.uint32), ref.w.view(np.uint32)), f"{what}: weights {l}"


@pytest.mark.parametrize("seed,n_nodes,n_edges,hi,weights", [
    (0, 1, 1, 1, "float"), (1, 10, 4, 3, "int"), (2, 50, 30, 5, "none"), (3, 300, 200, 8, "int"),
    (4, 1000, 700, 12, "float"), (5, 3000, 2500, 4, "int"), (6, 64, 300, 16, "float"), (7, 5000, 200, 60, "none"),
    (8, 20000, 15000, 30, "int"), (9, 257, 1000, 2, "none"),
    (10, 200000, 150000, 14, "int"), (11, 100000, 150000, 14, "float")])
def test_random_hypergraphs(oracle_mod, H, seed, n_nodes, n_edges, hi, weights):
    """Isolated nodes, singleton hyperedges, integer weights (many ties in
    the weight key, so size and id decide) and unit weights.  The last two
    have over 2^20 incidences, so the least rank per node is taken by
    bucketed minima (1024 and 512 nodes per bucket) instead of atomics."""
    hg = random_hypergraph(seed, n_nodes, n_edges, 1, hi, weighted=weights != "none",
                           integer_weights=weights == "int")
    _compare(oracle_mod, H, hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, hg.edge_w, 3,
             f"seed {seed}")


@pytest.mark.parametrize("name", ["tiny-2k", "hub-200k", "zipf-2m"])
def test_named_workload_hierarchy(oracle_mod, H, name):
    cfg = CONFIGS[name]
    hg = make_hypergraph(cfg)
    _compare(oracle_mod, H, hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, hg.edge_w, cfg.levels, name)


def test_friendster_scale_levels(oracle_mod, H):
    """8M nodes, 10M hyperedges, 125M incidences: the first step against the
    oracle, every step against the library's host coarsening (itself
    bit-exact with the oracle on the smaller workloads)."""
    cfg = CONFIGS["zipf-8m"]
    hg = make_hypergraph(cfg)
    _compare(oracle_mod, H, hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, hg.edge_w, 1, "zipf-8m")
    hier = H.Hierarchy.build(hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, hg.edge_w, cfg.levels)
    dev = H.Hierarchy.build(hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, hg.edge_w, cfg.levels, device="cuda")
    for l in range(cfg.levels):
        a, b = hier.maps[l], dev.maps[l]
        assert np.array_equal(a.node_rep, b.node_rep) and np.array_equal(a.edge_rep, b.edge_rep), f"step {l}"
        x, y = hier.levels[l + 1], dev.levels[l + 1]
        assert np.array_equal(x.edge_ptr, y.edge_ptr) and np.array_equal(x.edge_idx, y.edge_idx), f"level {l + 1}"


def test_no_hyperedges_and_empty(oracle_mod, H):
    import torch
    # nodes only: every node is a coarse node of its own
    lv = H.DeviceLevel(7, 0, 0, torch.zeros(1, dtype=torch.int32, device="cuda"),
                       torch.zeros(0, dtype=torch.int32, device="cuda"))
    nrep, erep, c = H.coarsen_level_device(lv)
    assert nrep.cpu().tolist() == list(range(7)) and erep.numel() == 0
    assert (c.n_nodes, c.n_edges, c.nnz) == (7, 0, 0) and c.edge_ptr.cpu().tolist() == [0]
    # nothing at all
    lv = H.DeviceLevel(0, 0, 0, torch.zeros(1, dtype=torch.int32, device="cuda"),
                       torch.zeros(0, dtype=torch.int32, device="cuda"))
    nrep, erep, c = H.coarsen_level_device(lv)
    assert (c.n_nodes, c.n_edges, c.nnz) == (0, 0, 0)
    # one hyperedge holding every node: it is removed, one coarse node is left
    n = 300
    lv = H.DeviceLevel(n, 1, n, torch.tensor([0, n], dtype=torch.int32, device="cuda"),
                       torch.arange(n, dtype=torch.int32, device="cuda"))
    nrep, erep, c = H.coarsen_level_device(lv)
    assert nrep.cpu().tolist() == [0] * n and erep.cpu().tolist() == [-1]
    assert (c.n_nodes, c.n_edges, c.nnz) == (1, 0, 0)


def test_dirty_workspace_and_reuse(oracle_mod, H):
    """Workspace contents are scratch: a workspace full of 0xFF, reused for
    two different levels in a row, gives the oracle's maps."""
    import torch
    O = oracle_mod
    big = random_hypergraph(11, 4000, 3000, 1, 9, weighted=True, integer_weights=True)
    small = random_hypergraph(12, 900, 500, 1, 6, weighted=False)
    ws = torch.full((H.coarsen_workspace_bytes(big.n_nodes, big.n_edges, big.nnz),), 255, dtype=torch.uint8,
                    device="cuda")
    for hg in (big, small, big):
        ref = O.coarsen_level(O.Level(hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, hg.edge_w))
        nrep, erep, c = H.coarsen_level_device(
            H.DeviceLevel.from_host(H.HostLevel(hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, hg.edge_w)), ws)
        assert np.array_equal(nrep.cpu().numpy(), ref.node_rep) and np.array_equal(erep.cpu().numpy(), ref.edge_rep)
        assert np.array_equal(c.edge_idx.cpu().numpy(), ref.coarse.eidx)


def _bad(H, n_nodes, ptr, idx, w=None):
    import torch
    lv = H.DeviceLevel(n_nodes, len(ptr) - 1, len(idx), torch.tensor(ptr, dtype=torch.int32, device="cuda"),
                       torch.tensor(idx, dtype=torch.int32, device="cuda"),
                       None if w is None else torch.tensor(w, dtype=torch.float32, device="cuda"))
    with pytest.raises(H.HnvError) as ei:
        H.coarsen_level_device(lv)
    return ei.value.status


def test_invalid_inputs_are_rejected(H):
    """The device-side check turns every malformed level into a status
    before any other kernel reads it (all reads stay inside the arrays)."""
    from paper_2103_09660_amd import _lib as L
    assert _bad(H, 4, [0, 2, 4], [0, 1, 3, 2]) == L.HNV_EUNSORTED
    assert _bad(H, 4, [0, 2, 4], [0, 1, 1, 1]) == L.HNV_EUNSORTED
    assert _bad(H, 4, [0, 2, 4], [0, 1, 2, 4]) == L.HNV_ERANGE
    assert _bad(H, 4, [0, 2, 4], [0, -1, 2, 3]) == L.HNV_ERANGE
    assert _bad(H, 4, [0, 2, 2, 4], [0, 1, 2, 3]) == L.HNV_EINVAL          # empty hyperedge
    assert _bad(H, 4, [0, 3, 2], [0, 1]) == L.HNV_EINVAL                    # decreasing offsets
    assert _bad(H, 4, [1, 2, 4], [0, 1, 2, 3]) == L.HNV_EINVAL              # does not start at 0
    assert _bad(H, 4, [0, 2, 3], [0, 1, 2, 3]) == L.HNV_EINVAL              # does not end at nnz
    assert _bad(H, 4, [0, 2, 4], [0, 1, 2, 3], [1.0, 0.0]) == L.HNV_EINVAL
    assert _bad(H, 4, [0, 2, 4], [0, 1, 2, 3], [1.0, float("nan")]) == L.HNV_EINVAL
    assert _bad(H, 4, [0, 2, 4], [0, 1, 2, 3], [float("inf"), 1.0]) == L.HNV_EINVAL
    assert _bad(H, 4, [3], []) == L.HNV_EINVAL                              # no hyperedges, offset not 0


def test_level_without_hyperedges(oracle_mod, H):
    """A level of nodes only: every node stays a node of its own, nothing else
    is written (the status of the same level with a bad offset is above)."""
    import torch
    O = oracle_mod
    lv = H.DeviceLevel(5, 0, 0, torch.zeros(1, dtype=torch.int32, device="cuda"),
                       torch.zeros(0, dtype=torch.int32, device="cuda"))
    nrep, erep, c = H.coarsen_level_device(lv)
    ref = O.coarsen_level(O.Level(5, 0, np.zeros(1, dtype=np.int64), np.zeros(0, dtype=np.int32), None))
    assert np.array_equal(nrep.cpu().numpy(), ref.node_rep)
    assert (c.n_nodes, c.n_edges, c.nnz) == (5, 0, 0)


def test_invalid_large_inputs_are_rejected(oracle_mod, H):
    """At the size where the least ranks are taken in LDS buckets (over 2^20
    incidences), malformed input reaches the step's later kernels, which read
    the check word first: the status comes back, and the same workspace then
    gives the oracle's maps for the valid level."""
    import torch
    from paper_2103_09660_amd import _lib as L
    O = oracle_mod
    hg = random_hypergraph(21, 300_000, 250_000, 1, 10, weighted=False)
    assert hg.nnz >= (1 << 20)
    ws = torch.empty(H.coarsen_workspace_bytes(hg.n_nodes, hg.n_edges, hg.nnz), dtype=torch.uint8, device="cuda")

    def run(ptr, idx):
        lv = H.DeviceLevel(hg.n_nodes, hg.n_edges, hg.nnz, torch.tensor(ptr, dtype=torch.int32, device="cuda"),
                           torch.tensor(idx, dtype=torch.int32, device="cuda"))
        return H.coarsen_level_device(lv, ws)

    ptr = hg.edge_ptr.astype(np.int32)
    e = int(np.argmax(np.diff(hg.edge_ptr) >= 2))
    last = int(hg.edge_ptr[e + 1]) - 1
    for k, (p2, i2, status) in enumerate([
            (ptr, np.where(np.arange(hg.nnz) == last, hg.n_nodes, hg.edge_idx), L.HNV_ERANGE),
            (ptr, np.where(np.arange(hg.nnz) == 7, -5, hg.edge_idx), L.HNV_ERANGE),
            (np.where(np.arange(hg.n_edges + 1) == hg.n_edges // 2, hg.nnz + 100, ptr), hg.edge_idx,
             L.HNV_EINVAL)]):
        with pytest.raises(H.HnvError) as ei:
            run(p2, i2.astype(np.int32))
        assert ei.value.status == status, k
    ref = O.coarsen_level(O.Level(hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, hg.edge_w))
    nrep, erep, c = run(ptr, hg.edge_idx.astype(np.int32))
    assert np.array_equal(nrep.cpu().numpy(), ref.node_rep) and np.array_equal(erep.cpu().numpy(), ref.edge_rep)
    assert np.array_equal(c.edge_idx.cpu().numpy(), ref.coarse.eidx)


def test_workspace_errors(H):
    import torch
    from paper_2103_09660_amd import _lib as L
    hg = random_hypergraph(3, 100, 60, 1, 5)
    lv = H.DeviceLevel.from_host(H.HostLevel(hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, hg.edge_w))
    need = H.coarsen_workspace_bytes(hg.n_nodes, hg.n_edges, hg.nnz)
    # the binding replaces a short workspace, so the statuses come from the C ABI itself
    import ctypes
    ws = torch.empty(need + 512, dtype=torch.uint8, device="cuda")
    out = [torch.empty(max(n, 1), dtype=dt, device="cuda") for n, dt in
           ((hg.n_nodes, torch.int32), (hg.n_edges, torch.int32), (hg.n_edges + 1, torch.int32),
            (hg.nnz, torch.int32), (hg.n_edges, torch.float32))]
    sizes = (ctypes.c_int64 * 3)()
    args = [hg.n_nodes, hg.n_edges, hg.nnz, lv.edge_ptr.data_ptr(), lv.edge_idx.data_ptr(), lv.edge_w.data_ptr()]
    args += [t.data_ptr() for t in out] + [ctypes.cast(sizes, L.i64p)]
    st = L.lib().hnv_coarsen_level_device(*args, ws.data_ptr(), need - 1, None)
    assert st == L.HNV_EWORKSPACE
    st = L.lib().hnv_coarsen_level_device(*args, ws.data_ptr() + 4, need, None)
    assert st == L.HNV_EWORKSPACE
    st = L.lib().hnv_coarsen_level_device(*args, ws.data_ptr(), need, None)
    assert st == L.HNV_OK and sizes[0] > 0


def test_depth_rule_matches_host(H):
    """The optional depth rule stops the GPU coarsening where it stops the
    host coarsening."""
    hg = random_hypergraph(5, 3000, 2000, 1, 6)
    full = H.Hierarchy.build(hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, hg.edge_w, 6)
    target = full.levels[3].rows
    host = H.Hierarchy.build(hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, hg.edge_w, 6, min_rows=target)
    dev = H.Hierarchy.build(hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, hg.edge_w, 6, device="cuda",
                            min_rows=target)
    assert host.n_levels == dev.n_levels == 4
    for a, b in zip(host.maps, dev.maps):
        assert np.array_equal(a.node_rep, b.node_rep) and np.array_equal(a.edge_rep, b.edge_rep)


def test_member_sort_boundaries(oracle_mod, H):
    """Coarse member lists sorted by a thread (up to 8 members by one network,
    up to 16 by another), a wavefront (up to 1,024, in 64-lane registers x
    1..16) or the library's segmented sort (longer): hyperedges at every
    boundary, with members whose coarse ids come out in every order, against
    the oracle bit for bit."""
    rng = np.random.default_rng(77)
    n_nodes = 6000
    sizes = [1, 2, 7, 8, 9, 12, 15, 16, 17, 63, 64, 65, 127, 128, 129, 255, 256, 257, 511, 512, 513, 1023, 1024,
             1025, 3000]
    sizes += list(rng.integers(2, 12, size=3000))      # small hyperedges that merge nodes into groups
    edges = [sorted(rng.choice(n_nodes, size=k, replace=False).tolist()) for k in sizes]
    ptr = np.concatenate([[0], np.cumsum([len(e) for e in edges])]).astype(np.int64)
    idx = np.array([v for e in edges for v in e], dtype=np.int32)
    _compare(oracle_mod, H, n_nodes, len(edges), ptr, idx, None, 2, "member sort boundaries")
