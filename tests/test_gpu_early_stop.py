"""Early stop decided on the device (Section 3.3's epsilon rule): a
refinement with tol > 0 enqueues every sweep and lets each sweep's
residual stage stop its level, so it must give, bit for bit, what a loop
driven from the host gives (single sweeps, each residual read back and
compared with tol): the same embedding, the same residuals packed in run
order, the same sweep counts.  It also runs inside a HIP graph.  Parity of
the early stop with the oracle is in test_gpu_parity.py."""
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


def _hier(H, seed, n, m, hi, steps):
    hg = random_hypergraph(seed, n, m, 1, hi, weighted=True)
    return H.Hierarchy.build(hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, hg.edge_w, steps)


def _host_driven(plan, zc, sweeps, omega, tol):
    """The reference: one sweep at a time, the residual read on the host."""
    import torch
    z, res, done = zc, [], [0] * plan.n_levels
    L = plan.n_levels - 1
    for l in range(L, -1, -1):
        if sweeps[l] == 0 and l < L:
            z = plan.project(l, z)
        for k in range(sweeps[l]):
            r = torch.zeros(1, dtype=torch.float64, device="cuda")
            z = plan.sweep(l, z, omega, from_coarse=(k == 0 and l < L), resid=r)
            res.append(r.item())
            done[l] += 1
            if r.item() <= tol:
                break
    return z, res, done


def _input(plan, seed):
    import torch
    g = torch.Generator().manual_seed(seed)
    return torch.randn(plan.rows(plan.n_levels - 1), plan.d, generator=g).to(plan.torch_dtype).cuda()


@pytest.mark.parametrize("dtype,order,d", [("f32", 0, 16), ("bf16", 0, 64), ("f32", 1, 32), ("bf16", 1, 128)])
def test_device_stop_equals_host_loop(H, dtype, order, d):
    import torch
    hier = _hier(H, 31, 3000, 2000, 12, 3)
    plan = H.Plan(hier, d, dtype, options={"order": order, "small_max": 8, "chunk": 64})
    zc = _input(plan, 1)
    # residual scale of this input, to place tol where levels stop at different sweeps
    r0 = torch.zeros(1, dtype=torch.float64, device="cuda")
    plan.sweep(plan.n_levels - 1, zc, 0.5, resid=r0)
    scale = r0.item()
    cases = [([30, 30, 30, 30], 0.05 * scale), ([8, 0, 12, 5], 0.2 * scale), ([1, 6, 0, 0], 0.5 * scale),
             ([25, 25, 25, 25], 1e-30), ([4, 4, 4, 4], 1e30), ([0, 3, 3, 3], 0.1 * scale)]
    for sweeps, tol in cases:
        ref, ref_res, ref_done = _host_driven(plan, zc, sweeps, 0.5, tol)
        out, res, done = plan.refine(zc, sweeps, 0.5, tol=tol, residuals=True)
        what = f"{dtype} order {order} sweeps {sweeps} tol {tol:.3g}"
        assert list(done) == ref_done, what
        assert torch.equal(out, ref), what
        got = res.cpu().numpy()
        assert np.array_equal(got[: len(ref_res)], np.array(ref_res)), what
        assert not got[len(ref_res):].any(), what          # entries past the last sweep run stay untouched
    # the counts are optional; the embedding does not depend on asking for them
    out2 = plan.refine(zc, [30, 30, 30, 30], 0.5, tol=cases[0][1])[0]
    assert torch.equal(out2, plan.refine(zc, [30, 30, 30, 30], 0.5, tol=cases[0][1], residuals=True)[0])


def test_levels_stop_independently(H):
    """A level stopped early does not stop the next: each level's first
    sweep runs, and a huge tol leaves exactly one sweep per level."""
    hier = _hier(H, 32, 2000, 1500, 8, 3)
    plan = H.Plan(hier, 32, "f32")
    zc = _input(plan, 2)
    _, _, done = plan.refine(zc, [5, 5, 5, 5], 0.5, tol=1e30)
    assert list(done) == [1, 1, 1, 1]
    _, _, done = plan.refine(zc, [5, 0, 5, 2], 0.5, tol=1e30)
    assert list(done) == [1, 0, 1, 1]
    _, _, done = plan.refine(zc, [5, 5, 5, 5], 0.5, tol=1e-300)
    assert list(done) == [5, 5, 5, 5]


def test_graph_replay_with_early_stop(H):
    """A refinement with tol captured into a HIP graph: every replay decides
    the stops anew and equals the eager call, also after the input has been
    refilled with data that stops the levels at other sweeps."""
    import torch
    hier = _hier(H, 33, 2500, 1800, 10, 3)
    plan = H.Plan(hier, 32, "f32")
    zc = _input(plan, 3)
    r0 = torch.zeros(1, dtype=torch.float64, device="cuda")
    plan.sweep(plan.n_levels - 1, zc, 0.5, resid=r0)
    tol = 0.1 * r0.item()
    sweeps = [20, 20, 20, 20]
    g = plan.capture_refine(zc, sweeps, 0.5, residuals=True, tol=tol)
    for seed, scale in ((3, 1.0), (4, 0.25), (5, 3.0), (3, 1.0)):
        zc.copy_(_input(plan, seed) * scale)
        ref, ref_res, ref_done = _host_driven(plan, zc.clone(), sweeps, 0.5, tol)
        out, res = g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, ref), f"seed {seed} scale {scale}"
        assert np.array_equal(res.cpu().numpy()[: len(ref_res)], np.array(ref_res)), f"seed {seed} scale {scale}"
        torch.cuda.synchronize()
