"""Stream semantics of the C ABI: every call enqueues its work on the
caller's stream (torch's current stream), so work on a side stream is
ordered after what that stream already holds, and plans on different
streams run side by side with the results each gives alone (no shared
state between plans; sweeps and reductions have a fixed order, so results
are bit-identical from run to run)."""
import numpy as np
import pytest

from tests.cases import random_hypergraph

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2103_09660_amd as H
    return H


def _plan(H, seed, n, m, hi, steps, d, dtype):
    hg = random_hypergraph(seed, n, m, 1, hi, weighted=True)
    hier = H.Hierarchy.build(hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, hg.edge_w, steps)
    return H.Plan(hier, d, dtype)


def _input(plan, seed):
    import torch
    g = torch.Generator().manual_seed(seed)
    return torch.randn(plan.rows(plan.n_levels - 1), plan.d, generator=g).to(plan.torch_dtype)


def test_refine_waits_for_its_stream(H):
    """The coarsest embedding is produced on a side stream behind a long
    matrix product; a refinement enqueued on that stream must read it only
    after it is written."""
    import torch
    plan = _plan(H, 21, 60000, 40000, 30, 2, 64, "f32")
    zc = _input(plan, 1)
    ref, _, _ = plan.refine(zc.cuda(), [4] * plan.n_levels)
    ref = ref.cpu()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        a = torch.randn(4096, 4096, device="cuda")
        slow = a @ a                                   # a few ms of work ahead of the input
        z = zc.cuda() + 0.0 * slow[0, 0]               # written only after the product
        out, _, _ = plan.refine(z, [4] * plan.n_levels)
    side.synchronize()
    assert torch.isfinite(slow[0, 0]).item()
    assert torch.equal(out.cpu(), ref)


def test_plans_on_separate_streams(H):
    """Two plans (BF16 and FP32, different hypergraphs) refined at the same
    time on two streams, and a reverse sweep of a third plan on a third
    stream, equal their results on the default stream bit for bit.  (One
    plan's calls share its scratch, so one plan is used on one stream at a
    time.)"""
    import torch
    pa = _plan(H, 22, 50000, 30000, 40, 3, 128, "bf16")
    pb = _plan(H, 23, 30000, 25000, 12, 2, 32, "f32")
    pc = H.Plan(pb.hier, 32, "f32")
    za, zb = _input(pa, 2).cuda(), _input(pb, 3).cuda()
    g = torch.randn(pb.rows(0), 32, generator=torch.Generator().manual_seed(4)).cuda()
    y = pb.empty(0).copy_(torch.randn(pb.rows(0), 32, generator=torch.Generator().manual_seed(5)))
    ra = pa.refine(za, [5] * pa.n_levels)[0].cpu()
    rb = pb.refine(zb, [5] * pb.n_levels)[0].cpu()
    zy = pc.sweep(0, y)
    ne = pc.level_info(0)[1]
    dw_ref = torch.zeros(ne, device="cuda")
    rg = pc.sweep_adjoint(0, g, y, zy, dw=dw_ref).cpu()
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream() for _ in range(3)]
    for s in streams:
        s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(streams[0]):
        oa = pa.refine(za, [5] * pa.n_levels)[0]
    with torch.cuda.stream(streams[1]):
        ob = pb.refine(zb, [5] * pb.n_levels)[0]
    with torch.cuda.stream(streams[2]):
        dw = torch.zeros(ne, device="cuda")
        og = pc.sweep_adjoint(0, g, y, zy, dw=dw)
    for s in streams:
        s.synchronize()
    assert torch.equal(oa.cpu(), ra)
    assert torch.equal(ob.cpu(), rb)
    assert torch.equal(og.cpu(), rg)
    assert torch.equal(dw.cpu(), dw_ref.cpu())


def test_device_coarsening_on_a_side_stream(H):
    """The GPU coarsening run on a side stream (while a refinement runs on
    another) gives the maps of a run on the default stream."""
    import torch
    hg = random_hypergraph(24, 40000, 30000, 1, 20, weighted=True, integer_weights=True)
    lv = H.DeviceLevel.from_host(H.HostLevel(hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, hg.edge_w))
    nrep, erep, c = H.coarsen_level_device(lv)
    ref = (nrep.cpu(), erep.cpu(), c.edge_idx.cpu())
    plan = _plan(H, 25, 50000, 30000, 40, 2, 64, "f32")
    z = _input(plan, 6).cuda()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    for s in (s1, s2):
        s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s1):
        plan.refine(z, [10] * plan.n_levels)
    with torch.cuda.stream(s2):
        n2, e2, c2 = H.coarsen_level_device(lv)
    s1.synchronize()
    s2.synchronize()
    assert torch.equal(n2.cpu(), ref[0]) and torch.equal(e2.cpu(), ref[1]) and torch.equal(c2.edge_idx.cpu(), ref[2])
