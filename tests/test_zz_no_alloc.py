"""hnv_sweep_noalloc, the sweep whose scratch is the library's static device
array, against hnv_sweep (scratch in the plan's workspace) through the C ABI:
the same kernels in the same order, so the outputs and residuals must be
identical bit for bit.  Two calls in a row, the second on a smaller input,
then a level too large for the static array (refused, while hnv_sweep still
serves it)."""
import numpy as np
import pytest

from tests.cases import random_hypergraph, tier_hypergraph

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2103_09660_amd as H
    return H


def _dev(x, dtype):
    import torch
    t = torch.as_tensor(np.ascontiguousarray(x, dtype=np.float32)).cuda()
    return t if dtype == "f32" else t.to(torch.bfloat16)


def _same(H, plan, level, z, from_coarse, what):
    """Runs both entry points on the same input and compares them."""
    import torch
    r_ws = torch.zeros(1, dtype=torch.float64, device="cuda")
    r_st = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
    want = plan.sweep(level, z, 0.5, from_coarse=from_coarse, resid=r_ws)
    got = plan.empty(level)
    got.fill_(7)                                # stale contents must not leak through
    plan.sweep_noalloc(level, z, 0.5, from_coarse=from_coarse, out=got, resid=r_st)
    torch.cuda.synchronize()
    assert torch.equal(got.view(torch.int16) if got.dtype == torch.bfloat16 else got.view(torch.int32),
                       want.view(torch.int16) if want.dtype == torch.bfloat16 else want.view(torch.int32)), what
    assert float(r_st.item()) == float(r_ws.item()), (what, float(r_st.item()), float(r_ws.item()))
    # without a residual
    got2 = plan.sweep_noalloc(level, z, 0.5, from_coarse=from_coarse)
    assert torch.equal(got2, want), what + " (no residual)"


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("order", ["jacobi", "edge_first"])
def test_noalloc_sweep_matches_workspace_sweep(H, dtype, order):
    import torch
    from paper_2103_09660_amd._lib import HNV_EUNSUPPORTED, HnvError
    print("no-alloc sweep", dtype, order, flush=True)
    # a hypergraph with rows on every tier, split rows included (chunk 64)
    hg = tier_hypergraph(3, 8, 64)
    hier = H.Hierarchy.build(hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, hg.edge_w, 2)
    plan = H.Plan(hier, 64, dtype, options={"small_max": 8, "chunk": 64, "order": order})
    rng = np.random.default_rng(5)
    n0, e0, _ = plan.level_info(0)
    n1, e1, _ = plan.level_info(1)
    z0 = _dev(rng.standard_normal((n0 + e0, 64)), dtype)
    z1 = _dev(rng.standard_normal((n1 + e1, 64)), dtype)
    # first call on the finest level, then a second on the smaller level 1
    _same(H, plan, 0, z0, False, f"{dtype} {order} level 0")
    _same(H, plan, 1, z1, False, f"{dtype} {order} level 1 (smaller, second call)")
    _same(H, plan, 0, z1, True, f"{dtype} {order} level 0 fused with the projection")
    # a second, smaller plan on the same array: a larger random hypergraph first
    big = random_hypergraph(8, 20000, 12000, 1, 300, weighted=True)
    hb = H.Hierarchy.build(big.n_nodes, big.n_edges, big.edge_ptr, big.edge_idx, big.edge_w, 1)
    pb = H.Plan(hb, 128, dtype, options={"chunk": 128, "order": order})
    nb, eb, _ = pb.level_info(0)
    _same(H, pb, 0, _dev(rng.standard_normal((nb + eb, 128)), dtype), False, f"{dtype} {order} larger plan")
    _same(H, plan, 1, z1, False, f"{dtype} {order} smaller plan after the larger one")
    if order == "edge_first":
        # in place within a level, as hnv_sweep allows for this order
        zi = z0.clone()
        want = plan.sweep(0, z0, 0.5)
        plan.sweep_noalloc(0, zi, 0.5, out=zi)
        assert torch.equal(zi, want)
    del pb
    torch.cuda.synchronize()


def test_noalloc_sweep_refuses_a_level_beyond_its_array(H):
    """d = 512 in FP32 and 32-neighbour chunks: every 64-member hyperedge is
    split into two partial slots of 520 floats, 40,000 of them need 166 MB of
    partial sums, more than the 64 MiB array."""
    import torch
    from paper_2103_09660_amd._lib import HNV_EUNSUPPORTED, HnvError, lib
    print("no-alloc refusal", flush=True)
    n_edges, size = 40000, 64
    n_nodes = 50000
    rng = np.random.default_rng(2)
    idx = np.sort(np.stack([rng.choice(n_nodes, size=size, replace=False) for _ in range(n_edges)]), axis=1)
    ptr = np.arange(n_edges + 1, dtype=np.int64) * size
    hier = H.Hierarchy.build(n_nodes, n_edges, ptr, idx.astype(np.int32).ravel(), None, 0)
    plan = H.Plan(hier, 512, "f32", options={"chunk": 32, "small_max": 1})
    z = _dev(rng.standard_normal((n_nodes + n_edges, 512)), "f32")
    with pytest.raises(HnvError) as ei:
        plan.sweep_noalloc(0, z, 0.5)
    assert ei.value.status == HNV_EUNSUPPORTED
    assert "scratch" in str(ei.value)
    out = plan.sweep(0, z, 0.5)                 # the workspace sweep still serves it
    torch.cuda.synchronize()
    assert bool(torch.isfinite(out).all())
