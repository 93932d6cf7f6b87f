"""A plan built on the GPU from device-resident levels against the plan built
on the host from the same levels: every result must be bit-identical
(same adjacency, same work lists in the same order, same reciprocals), and
the device-resident pipeline (GPU coarsening, GPU plan, refinement) must
match the FP64 oracle."""
import numpy as np
import pytest

from tests.cases import CONFIGS, assert_close, coarsest_embedding, make_hypergraph, random_hypergraph, tier_hypergraph

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2103_09660_amd as H
    return H


def _device_copy(H, hier):
    levels = [H.DeviceLevel.from_host(lv, "cuda") for lv in hier.levels]
    import torch
    maps = [(torch.as_tensor(m.node_rep).cuda(), torch.as_tensor(m.edge_rep).cuda()) for m in hier.maps]
    return levels, maps


def _both_plans(H, hier, d, dtype, options=None):
    levels, maps = _device_copy(H, hier)
    host = H.Plan(hier, d, dtype, options=options)
    dev = H.Plan.from_device(levels, maps, d, dtype, options=options)
    return host, dev


def _assert_same_refine(host, dev, hier, d, sweeps, seed):
    import torch
    zc = torch.as_tensor(coarsest_embedding(seed, hier.levels[-1].rows, d)).cuda().to(host.torch_dtype)
    a, ra, na = host.refine(zc, sweeps, 0.5, residuals=True)
    b, rb, nb = dev.refine(zc, sweeps, 0.5, residuals=True)
    torch.cuda.synchronize()
    assert torch.equal(a.view(torch.int16) if a.dtype == torch.bfloat16 else a.view(torch.int32),
                       b.view(torch.int16) if b.dtype == torch.bfloat16 else b.view(torch.int32))
    assert torch.equal(ra, rb) and np.array_equal(na, nb)
    for l in range(hier.n_levels):
        assert host.level_info(l) == dev.level_info(l)


@pytest.mark.parametrize("small_max,chunk", [(0, 0), (8, 16), (16, 64), (3, 5)])
@pytest.mark.parametrize("dtype,d,order", [("f32", 32, "jacobi"), ("bf16", 64, "jacobi"), ("f32", 128, "edge_first"),
                                           ("bf16", 16, "edge_first")])
def test_tiers_bit_identical(H, small_max, chunk, dtype, d, order):
    """Every tier on both sides, split rows on both sides, both orders."""
    sm, ch = (small_max or 64), (chunk or 512)
    hg = tier_hypergraph(7, sm, ch)
    hier = H.Hierarchy.build(hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, hg.edge_w, 2)
    opts = {"small_max": small_max, "chunk": chunk, "order": order}
    host, dev = _both_plans(H, hier, d, dtype, opts)
    _assert_same_refine(host, dev, hier, d, [3, 2, 2], 11)


@pytest.mark.parametrize("n_edges", [1, 63, 64, 65, 127, 128, 129, 191])
def test_side_boundary_bit_identical(H, n_edges):
    """Both sides' degree tiers are built over one array of entries in which
    side 1 starts at the first multiple of 64 past side 0's rows: hyperedge
    counts on either side of those multiples, with split rows on both sides
    (small_max 4, chunk 8) and with the default tiers."""
    n_nodes = max(64, 3 * n_edges + 5)
    hg = random_hypergraph(100 + n_edges, n_nodes, n_edges, 1, 40)
    hier = H.Hierarchy.build(hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, hg.edge_w, 2)
    for opts in ({"small_max": 4, "chunk": 8}, None):
        host, dev = _both_plans(H, hier, 32, "f32", opts)
        _assert_same_refine(host, dev, hier, 32, [2, 2, 2][:hier.n_levels], 5)


@pytest.mark.parametrize("seed,n_nodes,n_edges,hi,weighted", [
    (0, 40, 20, 4, True), (1, 3000, 2000, 12, False), (2, 700, 900, 40, True), (3, 1, 1, 1, False)])
def test_random_bit_identical(H, seed, n_nodes, n_edges, hi, weighted):
    hg = random_hypergraph(seed, n_nodes, n_edges, 1, hi, weighted=weighted)
    hier = H.Hierarchy.build(hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, hg.edge_w, 3)
    host, dev = _both_plans(H, hier, 24, "f32")
    _assert_same_refine(host, dev, hier, 24, [2, 2, 2, 2], seed)


@pytest.mark.parametrize("order", ["jacobi", "edge_first"])
def test_reverse_bit_identical(H, order):
    """Adjoint sweep, weight gradient and projection adjoint through both plans."""
    import torch
    cfg = CONFIGS["hub-200k"]
    hg = make_hypergraph(cfg)
    hier = H.Hierarchy.build(hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, hg.edge_w, 1)
    host, dev = _both_plans(H, hier, 32, "f32", options={"order": order})
    rng = np.random.default_rng(3)
    y = torch.as_tensor(rng.standard_normal((hier.levels[0].rows, 32)).astype(np.float32)).cuda()
    g = torch.as_tensor(rng.standard_normal((hier.levels[0].rows, 32)).astype(np.float32)).cuda()
    outs = []
    for p in (host, dev):
        z = p.sweep(0, y, 0.5)
        dw = torch.zeros(hier.levels[0].n_edges, dtype=torch.float32, device="cuda")
        gy = p.sweep_adjoint(0, g, y, z, 0.5, dw=dw)
        gc = p.project_adjoint(0, gy)
        outs.append((z, gy, dw, gc))
    torch.cuda.synchronize()
    for a, b in zip(*outs):
        assert torch.equal(a.view(torch.int32), b.view(torch.int32))


@pytest.mark.parametrize("name", ["hub-200k", "zipf-2m"])
def test_device_pipeline_bit_identical(H, name):
    """GPU coarsening -> GPU plan -> refinement equals host coarsening ->
    host plan -> refinement, bit for bit, at full size."""
    import torch
    cfg = CONFIGS[name]
    hg = make_hypergraph(cfg)
    hier = H.Hierarchy.build(hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, hg.edge_w, cfg.levels)
    lv0 = H.DeviceLevel.from_host(hier.levels[0], "cuda")
    dl, dm = H.coarsen_hierarchy_device(lv0, cfg.levels)
    dtype = cfg.dtypes[0]
    host = H.Plan(hier, cfg.d, dtype)
    dev = H.Plan.from_device(dl, dm, cfg.d, dtype)
    _assert_same_refine(host, dev, hier, cfg.d, list(cfg.sweeps), cfg.seed)
    del host, dev
    torch.cuda.empty_cache()


def test_device_pipeline_vs_oracle(oracle_mod, H):
    import torch
    O = oracle_mod
    cfg = CONFIGS["tiny-2k"]
    hg = make_hypergraph(cfg)
    levels, maps = O.build_hierarchy(hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, hg.edge_w, cfg.levels)
    lv0 = H.DeviceLevel.from_host(H.HostLevel(hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, hg.edge_w), "cuda")
    dl, dm = H.coarsen_hierarchy_device(lv0, cfg.levels)
    plan = H.Plan.from_device(dl, dm, cfg.d, "f32")
    zc = coarsest_embedding(cfg, levels[-1].rows, cfg.d)
    out, _, _ = plan.refine(torch.as_tensor(zc).cuda(), list(cfg.sweeps), 0.5)
    ref = O.refine(levels, maps, zc, list(cfg.sweeps), 0.5)
    assert_close(out.cpu().numpy(), ref, 1e-5, "device pipeline vs oracle")


def test_device_plan_checks(H):
    """The device-side checks report the host statuses."""
    import torch
    from paper_2103_09660_amd import _lib as L
    hg = random_hypergraph(4, 200, 120, 1, 6)
    hier = H.Hierarchy.build(hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, hg.edge_w, 1)
    levels, maps = _device_copy(H, hier)
    # node map out of range
    bad = maps[0][0].clone()
    bad[5] = hier.levels[1].n_nodes
    with pytest.raises(H.HnvError) as ei:
        H.Plan.from_device(levels, [(bad, maps[0][1])], 16, "f32")
    assert ei.value.status == L.HNV_ERANGE
    # hyperedge map out of range
    bad = maps[0][1].clone()
    bad[0] = hier.levels[1].n_edges
    with pytest.raises(H.HnvError) as ei:
        H.Plan.from_device(levels, [(maps[0][0], bad)], 16, "f32")
    assert ei.value.status == L.HNV_ERANGE
    # unsorted members: rejected with validation, accepted without (as on the host)
    idx = levels[0].edge_idx.clone()
    e = int(np.nonzero(np.diff(hg.edge_ptr) >= 2)[0][0])
    a = int(hg.edge_ptr[e])
    idx[a], idx[a + 1] = int(idx[a + 1]), int(idx[a])
    lv = H.DeviceLevel(levels[0].n_nodes, levels[0].n_edges, levels[0].nnz, levels[0].edge_ptr, idx,
                       levels[0].edge_w)
    with pytest.raises(H.HnvError) as ei:
        H.Plan.from_device([lv], [], 16, "f32")
    assert ei.value.status == L.HNV_EUNSORTED
    H.Plan.from_device([lv], [], 16, "f32", validate=False)
    # member out of range: always rejected
    idx = levels[0].edge_idx.clone()
    idx[3] = levels[0].n_nodes
    lv = H.DeviceLevel(levels[0].n_nodes, levels[0].n_edges, levels[0].nnz, levels[0].edge_ptr, idx,
                       levels[0].edge_w)
    with pytest.raises(H.HnvError) as ei:
        H.Plan.from_device([lv], [], 16, "f32", validate=False)
    assert ei.value.status == L.HNV_ERANGE
    # offsets out of range and decreasing: rejected with or without
    # validation; the build, which runs before the plan's single read-back,
    # writes placeholder arrays for such a level instead of following them
    for vflag in (True, False):
        ptr = levels[0].edge_ptr.clone()
        ptr[2] = levels[0].nnz + 7
        lv = H.DeviceLevel(levels[0].n_nodes, levels[0].n_edges, levels[0].nnz, ptr, levels[0].edge_idx,
                           levels[0].edge_w)
        with pytest.raises(H.HnvError) as ei:
            H.Plan.from_device([lv, levels[1]], [maps[0]], 16, "f32", validate=vflag)
        assert ei.value.status == L.HNV_EINVAL
    torch.cuda.synchronize()
    # non-positive weight: rejected with validation
    w = levels[0].edge_w.clone()
    w[2] = 0.0
    lv = H.DeviceLevel(levels[0].n_nodes, levels[0].n_edges, levels[0].nnz, levels[0].edge_ptr,
                       levels[0].edge_idx, w)
    with pytest.raises(H.HnvError) as ei:
        H.Plan.from_device([lv], [], 16, "f32")
    assert ei.value.status == L.HNV_EINVAL
    # a coarser level with more rows than the finest (a valid map onto a
    # level with unused nodes) does not fit the refinement's buffers
    big = H.DeviceLevel.from_host(H.HostLevel(hier.levels[0].rows + 5, 1, np.array([0, 1], np.int64),
                                              np.array([0], np.int32), None), "cuda")
    with pytest.raises(H.HnvError) as ei:
        H.Plan.from_device([levels[0], big], [(torch.zeros_like(maps[0][0]), torch.full_like(maps[0][1], -1))],
                           16, "f32")
    assert ei.value.status == L.HNV_EUNSUPPORTED
    torch.cuda.synchronize()


def test_documented_usage_flow(H):
    """The usage shown in the README, at a small size: device pipeline in
    BF16, then a differentiable finest-level refinement in FP32."""
    import torch
    cfg = CONFIGS["tiny-2k"]
    hg = make_hypergraph(cfg)
    lv0 = H.DeviceLevel.from_host(H.HostLevel(hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, hg.edge_w))
    levels, maps = H.coarsen_hierarchy_device(lv0, cfg.levels)
    plan = H.Plan.from_device(levels, maps, d=32, dtype="bf16")
    z_coarse = H.cast(torch.randn(levels[-1].n_nodes + levels[-1].n_edges, 32, device="cuda"), "bf16")
    z_fine, residuals, done = plan.refine(z_coarse, sweeps=[5] * plan.n_levels, omega=0.5, residuals=True)
    assert z_fine.shape == (levels[0].n_nodes + levels[0].n_edges, 32) and list(done) == [5] * plan.n_levels
    assert bool(torch.isfinite(residuals).all())
    plan32 = H.Plan.from_device(levels, maps, d=32, dtype="f32")
    theta = torch.zeros(levels[0].n_edges, device="cuda", requires_grad=True)
    z1 = torch.randn(levels[1].n_nodes + levels[1].n_edges, 32, device="cuda", requires_grad=True)
    z0 = H.refine_level(z1, theta, plan32, 0, 10, 0.5, from_coarse=True, ckpt_every=5)
    z0[: levels[0].n_nodes].square().mean().backward()
    assert theta.grad is not None and z1.grad is not None
    assert bool(torch.isfinite(theta.grad).all()) and float(z1.grad.abs().sum()) > 0


def test_plan_build_option(H):
    """Plan(hierarchy, build="device") uploads the host levels and gives the
    plan hnv_plan_create builds, bit for bit."""
    cfg = CONFIGS["hub-200k"]
    hg = make_hypergraph(cfg)
    hier = H.Hierarchy.build(hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, hg.edge_w, cfg.levels)
    host = H.Plan(hier, cfg.d, "bf16")
    dev = H.Plan(hier, cfg.d, "bf16", build="device")
    _assert_same_refine(host, dev, hier, cfg.d, list(cfg.sweeps), 2)
    with pytest.raises(ValueError):
        H.Plan(hier, cfg.d, "bf16", build="somewhere")


@pytest.mark.parametrize("dtype,d", [("bf16", 128), ("f32", 64), ("f32", 256), ("bf16", 8)])
def test_device_score_plan_bit_identical(H, dtype, d):
    """Candidates planned on the GPU give the host score plan's features bit
    for bit, for every statistic; candidates include empty ones and ones long
    enough to split."""
    import torch
    rng = np.random.default_rng(d)
    n_nodes = 5000
    sizes = np.concatenate([rng.integers(0, 6, 3000), rng.integers(60, 200, 50), [0, 1, 1500, 600]])
    ptr = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    idx = rng.integers(0, n_nodes, int(ptr[-1])).astype(np.int32)
    z = torch.randn(n_nodes, d, device="cuda").to(torch.float32 if dtype == "f32" else torch.bfloat16)
    host = H.ScorePlan(ptr, idx, n_nodes, d, dtype)
    dev = H.ScorePlan.from_device(torch.as_tensor(ptr.astype(np.int32)).cuda(), torch.as_tensor(idx).cuda(),
                                  n_nodes, d, dtype)
    for op in ("variance", "mean", "min", "max"):
        a, b = host.score(z, op), dev.score(z, op)
        torch.cuda.synchronize()
        assert torch.equal(a.view(torch.int32), b.view(torch.int32)), op


def test_device_score_plan_checks(H):
    import torch
    from paper_2103_09660_amd import _lib as L
    ptr = torch.tensor([0, 2, 5], dtype=torch.int32, device="cuda")
    with pytest.raises(H.HnvError) as ei:
        H.ScorePlan.from_device(ptr, torch.tensor([0, 1, 2, 9, 3], dtype=torch.int32, device="cuda"), 9, 16)
    assert ei.value.status == L.HNV_ERANGE
    with pytest.raises(H.HnvError) as ei:
        H.ScorePlan.from_device(torch.tensor([0, 3, 2], dtype=torch.int32, device="cuda"),
                                torch.tensor([0, 1], dtype=torch.int32, device="cuda"), 9, 16)
    assert ei.value.status == L.HNV_EINVAL
    # no candidates at all
    p = H.ScorePlan.from_device(torch.zeros(1, dtype=torch.int32, device="cuda"),
                                torch.zeros(0, dtype=torch.int32, device="cuda"), 9, 16)
    assert p.score(torch.zeros(9, 16, device="cuda")).shape == (0, 16)
