"""The device calls of the C ABI reject bad arguments with the documented
status codes (no kernel is launched for them), and the kernel-timing hook
counts every sweep launch."""
import numpy as np
import pytest

from tests.cases import random_hypergraph

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2103_09660_amd as H
    hg = random_hypergraph(3, 300, 200, 1, 8, weighted=True)
    hier = H.Hierarchy.build(hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, hg.edge_w, 2)
    plan = H.Plan(hier, 32, "f32")
    return H, torch, hier, plan


def _status(fn):
    from paper_2103_09660_amd._lib import HnvError
    with pytest.raises(HnvError) as ei:
        fn()
    return ei.value.status


def test_device_call_argument_errors(setup):
    from paper_2103_09660_amd import _lib as L
    H, torch, hier, plan = setup
    z0 = plan.empty(0).normal_()
    s = torch.cuda.current_stream().cuda_stream
    lib = L.lib()
    # aliasing, omega out of range, level out of range, from_coarse at the coarsest level
    assert lib.hnv_sweep(plan._h, 0, z0.data_ptr(), z0.data_ptr(), 0.5, 0, None, s) == L.HNV_EINVAL
    assert lib.hnv_sweep(plan._h, 0, z0.data_ptr(), plan.empty(0).data_ptr(), 1.5, 0, None, s) == L.HNV_EINVAL
    assert lib.hnv_sweep(plan._h, 5, z0.data_ptr(), plan.empty(0).data_ptr(), 0.5, 0, None, s) == L.HNV_EINVAL
    z2 = plan.empty(2)
    assert lib.hnv_sweep(plan._h, 2, z2.data_ptr(), plan.empty(2).data_ptr(), 0.5, 1, None, s) == L.HNV_EINVAL
    # misaligned pointer
    raw = torch.empty(plan.rows(0) * 32 + 4, device="cuda")
    assert lib.hnv_sweep(plan._h, 0, raw.data_ptr() + 4, z0.data_ptr(), 0.5, 0, None, s) == L.HNV_EINVAL
    assert "aligned" in H.last_error()
    # reverse sweep needs omega > 0
    g = plan.empty(0).normal_()
    assert lib.hnv_sweep_adjoint(plan._h, 0, g.data_ptr(), plan.empty(0).data_ptr(), z0.data_ptr(),
                                 z0.data_ptr(), None, 0.0, s) == L.HNV_EINVAL
    # projection adjoint at the coarsest level, refine with aliased buffers, negative sweep count
    assert lib.hnv_project_adjoint(plan._h, 2, z2.data_ptr(), z2.data_ptr(), s) == L.HNV_EINVAL
    sw = np.array([1, 1, 1], dtype=np.int32)
    assert lib.hnv_refine(plan._h, z0.data_ptr(), z0.data_ptr(), sw.ctypes.data_as(L.i32p), 0.5, 0.0,
                          None, None, s) == L.HNV_EINVAL
    sw_bad = np.array([1, -1, 1], dtype=np.int32)
    assert lib.hnv_refine(plan._h, z2.data_ptr(), z0.data_ptr(), sw_bad.ctypes.data_as(L.i32p), 0.5, 0.0,
                          None, None, s) == L.HNV_EINVAL
    # the binding checks shapes and dtypes before calling
    with pytest.raises(ValueError):
        plan.sweep(0, z0.to(torch.bfloat16), 0.5)
    with pytest.raises(ValueError):
        plan.sweep(0, z0[:-1], 0.5)
    torch.cuda.synchronize()


def test_workspace_and_plan_errors(setup):
    from paper_2103_09660_amd import _lib as L
    import ctypes
    H, torch, hier, plan = setup
    lv, mp = hier.c_arrays()
    need = H.plan_workspace_bytes(hier, 32, "f32")
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    out = ctypes.c_void_p()
    s = torch.cuda.current_stream().cuda_stream
    st = L.lib().hnv_plan_create(lv, mp, hier.n_levels, 32, L.HNV_F32, None, 1, ws.data_ptr(), need - 256, s,
                                 ctypes.byref(out))
    assert st == L.HNV_EWORKSPACE and not out.value
    st = L.lib().hnv_plan_create(lv, mp, hier.n_levels, 32, L.HNV_F32, None, 1, ws.data_ptr() + 16, need, s,
                                 ctypes.byref(out))
    assert st == L.HNV_EWORKSPACE
    # a map entry out of range is caught even without full validation
    bad = H.HostMap(hier.maps[0].node_rep.copy(), hier.maps[0].edge_rep.copy())
    bad.node_rep[3] = hier.levels[1].n_nodes
    h2 = H.Hierarchy(hier.levels, [bad, hier.maps[1]])
    lv2, mp2 = h2.c_arrays()
    st = L.lib().hnv_plan_create(lv2, mp2, h2.n_levels, 32, L.HNV_F32, None, 0, ws.data_ptr(), need, s,
                                 ctypes.byref(out))
    assert st == L.HNV_ERANGE


def test_profiling_counts_launches(setup):
    H, torch, hier, plan = setup
    zc = plan.empty(2).normal_()
    plan.set_profiling(True)
    plan.refine(zc, [2, 3, 4], 0.5)
    n_sweep, ms = plan.profile_read(0)      # non-fused forward sweeps
    n_fused, _ = plan.profile_read(1)
    assert (n_sweep, n_fused) == (4 + 2 + 1, 2) and ms > 0      # level 2: 4; level 1: 1 fused + 2; level 0: 1 + 1
    assert plan.profile_read(0, 2)[0] == 4
    plan.set_profiling(False)
    assert plan.profile_read(0)[0] == 0


def test_binding_checks_vectors_before_calling(setup):
    """Every device vector a kernel reads or writes is checked for type,
    contiguity and length by the binding, so a short tensor is a ValueError
    and never an out-of-bounds access."""
    H, torch, hier, plan = setup
    ne = plan.level_info(0)[1]
    f32 = dict(dtype=torch.float32, device="cuda")
    with pytest.raises(ValueError):
        plan.set_edge_weights(0, torch.ones(ne - 1, **f32))
    with pytest.raises(ValueError):
        plan.set_edge_weights(0, torch.ones(ne, dtype=torch.float64, device="cuda"))
    with pytest.raises(ValueError):
        plan.set_edge_logweights(0, torch.zeros(2 * ne, **f32)[::2])
    with pytest.raises(ValueError):
        plan.set_edge_logweights(0, torch.zeros(ne, **f32), w_out=torch.zeros(ne - 1, **f32))
    with pytest.raises(ValueError):
        plan.logweight_grad(0, torch.zeros(ne, **f32), torch.zeros(1, **f32))
    z0 = plan.empty(0).normal_()
    with pytest.raises(ValueError):
        plan.sweep(0, z0, resid=torch.zeros(1, **f32))
    with pytest.raises(ValueError):
        plan.sweep_adjoint(0, z0, z0, z0, dw=torch.zeros(ne - 1, **f32))
    with pytest.raises(ValueError):
        plan.refine(plan.empty(plan.n_levels - 1), [1] * (plan.n_levels + 1))
    sp = H.ScorePlan(np.array([0, 2, 3]), np.array([0, 5, 7], dtype=np.int32), 10, 32)
    with pytest.raises(ValueError):
        sp.score(torch.zeros(9, 32, **f32))                        # fewer rows than the plan's ids need
    with pytest.raises(ValueError):
        sp.score(torch.zeros(10, 32, **f32), out=torch.empty(1, 32, **f32))
    lv = H.DeviceLevel(4, 2, 4, torch.tensor([0, 2, 4], dtype=torch.int32, device="cuda"),
                       torch.tensor([0, 1, 2], dtype=torch.int32, device="cuda"))   # one member short
    with pytest.raises(ValueError):
        H.coarsen_level_device(lv)
    # valid vectors still pass (the level's own weights, so the shared plan is unchanged)
    plan.set_edge_weights(0, torch.as_tensor(hier.levels[0].edge_w).cuda())
    assert torch.isfinite(sp.score(torch.ones(10, 32, **f32))).all()


def test_plan_from_a_caller_csc(setup):
    """A level that carries its own CSC (node -> hyperedges) gives the plan
    the derived CSC gives, hence a bit-identical refinement and reverse
    sweep; a CSC that is not the transpose is refused at plan creation."""
    import dataclasses
    from paper_2103_09660_amd._lib import HNV_EINVAL, HnvError
    H, torch, hier, plan = setup
    lv0 = hier.levels[0]
    order = np.argsort(lv0.edge_idx, kind="stable")          # incidences by node, hyperedges ascending
    e_of = np.repeat(np.arange(lv0.n_edges, dtype=np.int32), np.diff(lv0.edge_ptr))
    nptr = np.concatenate([[0], np.cumsum(np.bincount(lv0.edge_idx, minlength=lv0.n_nodes))]).astype(np.int64)
    nidx = e_of[order]
    with_csc = H.Hierarchy([dataclasses.replace(lv0, node_ptr=nptr, node_idx=nidx)] + hier.levels[1:], hier.maps)
    p2 = H.Plan(with_csc, 32, "f32")
    zc = torch.randn((hier.levels[-1].rows, 32), device="cuda")
    a, _, _ = plan.refine(zc, [2, 2, 2], 0.5)
    b, _, _ = p2.refine(zc, [2, 2, 2], 0.5)
    assert torch.equal(a, b)
    g = torch.randn_like(a)
    dw1 = torch.zeros(lv0.n_edges, device="cuda")
    dw2 = torch.zeros(lv0.n_edges, device="cuda")
    z1 = plan.sweep(0, a, 0.5)
    assert torch.equal(plan.sweep_adjoint(0, g, a, z1, 0.5, dw=dw1), p2.sweep_adjoint(0, g, a, z1, 0.5, dw=dw2))
    assert torch.equal(dw1, dw2)
    bad = nidx.copy()
    bad[0] = (bad[0] + 1) % lv0.n_edges
    with pytest.raises(HnvError) as ei:
        H.Plan(H.Hierarchy([dataclasses.replace(lv0, node_ptr=nptr, node_idx=bad)] + hier.levels[1:], hier.maps),
               32, "f32")
    assert ei.value.status == HNV_EINVAL
    torch.cuda.synchronize()

