"""Refinement captured into a HIP graph (through torch.cuda.CUDAGraph):
every launch of hnv_refine without early stop or profiling is a kernel on
the caller's stream, so the whole multi-level refinement can be replayed
from a graph.  Each replay, with eager work and synchronisations between
replays, must equal the eager result bit for bit."""
import numpy as np
import pytest

from tests.cases import CONFIGS, coarsest_embedding, make_hypergraph

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2103_09660_amd as H
    return H


@pytest.mark.parametrize("dtype,order", [("f32", "jacobi"), ("bf16", "jacobi"), ("f32", "edge_first")])
def test_refine_replays_from_a_graph(H, dtype, order):
    import torch
    cfg = CONFIGS["tiny-2k"]
    hg = make_hypergraph(cfg)
    hier = H.Hierarchy.build(hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, hg.edge_w, cfg.levels)
    plan = H.Plan(hier, cfg.d, dtype, options={"order": order})
    zc = torch.as_tensor(coarsest_embedding(cfg, hier.levels[-1].rows, cfg.d)).cuda().to(plan.torch_dtype)
    sweeps = list(cfg.sweeps)
    eager, eager_res, _ = plan.refine(zc, sweeps, 0.5, residuals=True)
    torch.cuda.synchronize()
    out = plan.empty(0)
    res = torch.zeros(int(sum(sweeps)), dtype=torch.float64, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):          # warm-up on the capture stream
        plan.refine(zc, sweeps, 0.5, out=out)
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        import ctypes
        from paper_2103_09660_amd import _lib as L
        sw = np.ascontiguousarray(sweeps, dtype=np.int32)
        done = np.zeros(len(sweeps), dtype=np.int32)
        L.call("hnv_refine", plan._h, zc.data_ptr(), out.data_ptr(), sw.ctypes.data_as(L.i32p), 0.5, 0.0,
               res.data_ptr(), done.ctypes.data_as(L.i32p), torch.cuda.current_stream().cuda_stream)
    for i in range(3):
        out.zero_()
        res.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        a = out.view(torch.int16) if out.dtype == torch.bfloat16 else out.view(torch.int32)
        b = eager.view(torch.int16) if eager.dtype == torch.bfloat16 else eager.view(torch.int32)
        assert torch.equal(a, b), f"replay {i}"
        assert torch.equal(res, eager_res), f"replay {i} residuals"
        # eager work between replays
        plan.refine(zc, sweeps, 0.5)
        torch.cuda.synchronize()


def test_capture_refine_api(H):
    """Plan.capture_refine: replays equal eager refinement bit for bit and
    follow the refilled input."""
    import torch
    cfg = CONFIGS["tiny-2k"]
    hg = make_hypergraph(cfg)
    hier = H.Hierarchy.build(hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, hg.edge_w, cfg.levels)
    plan = H.Plan(hier, cfg.d, "bf16")
    rows = hier.levels[-1].rows
    zc = torch.empty((rows, cfg.d), dtype=torch.bfloat16, device="cuda")
    g = plan.capture_refine(zc, list(cfg.sweeps), 0.5, residuals=True)
    for seed in (1, 2, 3):
        zc.copy_(torch.as_tensor(coarsest_embedding(seed, rows, cfg.d)).to(torch.bfloat16))
        out, res = g.replay()
        ref, ref_res, _ = plan.refine(zc, list(cfg.sweeps), 0.5, residuals=True)
        torch.cuda.synchronize()
        assert torch.equal(out.view(torch.int16), ref.view(torch.int16)) and torch.equal(res, ref_res)
