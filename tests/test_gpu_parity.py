"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs.  Tolerances hold element by element,
|got - ref| <= tol (|ref| + rms(ref)), and for the Frobenius norm of the
difference: FP32 storage tol = 1e-5; BF16 storage tol = 1e-2 against the
oracle run on the BF16-rounded input; reverse mode in FP32 tol = 1e-4.  The
BF16 reverse mode (cotangents and the hyperedge-weight gradient) is held to
twice a first-order rounding bound derived per element
(``tests.cases.bf16_reverse_bounds``) plus the FP32 tolerance."""
import numpy as np
import pytest

from tests.cases import (CONFIGS, assert_bf16, assert_close, assert_within, bf16_reverse_bounds, both_hierarchies,
                         coarsest_embedding, make_hypergraph, oracle_refine_bf16, oracle_sweep_bf16, random_hypergraph,
                         rel_fro, tier_hypergraph)

pytestmark = pytest.mark.gpu

F32_TOL = 1e-5
BF16_TOL = 1e-2
GRAD_TOL = 1e-4


@pytest.fixture(scope="module")
def H():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2103_09660_amd as H
    return H


def _dev(x, dtype="f32"):
    import torch
    t = torch.as_tensor(np.ascontiguousarray(x, dtype=np.float32)).cuda()
    return t if dtype == "f32" else t.to(torch.bfloat16)


def _host(t):
    import torch
    return t.float().cpu().numpy().astype(np.float64) if t.dtype != torch.float64 else t.cpu().numpy()


def _bf16_round(x):
    import torch
    return torch.as_tensor(np.asarray(x, dtype=np.float32)).to(torch.bfloat16).float().numpy().astype(np.float64)


def _assert_close(got, ref, tol, what):
    """tol per element and norm-wise (FP32 storage, reverse mode in FP32)."""
    assert_close(got, ref, tol, what)


def _floor(ref, tol):
    ref = np.asarray(ref, dtype=np.float64)
    return tol * (np.abs(ref) + np.sqrt(np.mean(ref * ref)))


def _assert_bf16_reverse(O, lv, ys, zs, g_top, omega, w, order, g_got, g_ref, dw_got, dw_ref, what):
    """BF16 reverse sweeps: twice the first-order rounding bound of every
    element plus the FP32 tolerance (the arithmetic itself)."""
    Eg, Bdw = bf16_reverse_bounds(O, lv, ys, zs, g_top, omega, w, order)
    if g_got is not None:
        assert_within(g_got, g_ref, 2 * Eg + _floor(g_ref, F32_TOL), f"{what} cotangent")
    if dw_got is not None:
        assert_within(dw_got, dw_ref, 2 * Bdw + _floor(dw_ref, GRAD_TOL), f"{what} dL/dw")


# ---------------------------------------------------------------------------
# single sweeps over random hypergraphs and every tier
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed,n_nodes,n_edges,d,weighted", [
    (0, 50, 30, 8, True), (1, 300, 200, 32, False), (2, 1000, 700, 40, True),
    (3, 2000, 900, 64, True), (4, 513, 129, 128, False), (5, 64, 300, 16, True),
    (6, 900, 600, 256, True), (7, 100, 80, 512, False)])
def test_sweep_and_fused_projection(oracle_mod, H, seed, n_nodes, n_edges, d, weighted):
    import torch
    O = oracle_mod
    hg = random_hypergraph(seed, n_nodes, n_edges, 1, 12, weighted=weighted)
    levels, maps, hier = both_hierarchies(O, H, hg, 1)
    plan = H.Plan(hier, d, "f32")
    rng = np.random.default_rng(seed)
    z0 = rng.standard_normal((levels[0].rows, d)).astype(np.float32)
    zc = rng.standard_normal((levels[1].rows, d)).astype(np.float32)
    resid = torch.zeros(1, dtype=torch.float64, device="cuda")
    for omega in (0.5, 0.3, 1.0):
        out = _host(plan.sweep(0, _dev(z0), omega, resid=resid))
        ref = O.sweep(levels[0], z0, omega)
        _assert_close(out, ref, F32_TOL, f"sweep omega={omega}")
        assert abs(float(resid.item()) - O.residual(ref, z0)) <= 1e-5 * max(1.0, O.residual(ref, z0))
        fused = _host(plan.sweep(0, _dev(zc), omega, from_coarse=True))
        ref_f = O.sweep(levels[0], O.project(O.rowmap(levels[0], maps[0]), zc), omega)
        _assert_close(fused, ref_f, F32_TOL, f"fused omega={omega}")
    proj = _host(plan.project(0, _dev(zc)))
    np.testing.assert_array_equal(proj, O.project(O.rowmap(levels[0], maps[0]), zc))
    # full-width FP32 rows (one pass, 32 B per lane from 128 columns up)
    full = H.Plan(hier, d, "f32", options={"panel_cols": d})
    _assert_close(_host(full.sweep(0, _dev(z0), 0.5)), O.sweep(levels[0], z0, 0.5), F32_TOL, "full-width sweep")
    _assert_close(_host(full.sweep(0, _dev(zc), 0.5, from_coarse=True)),
                  O.sweep(levels[0], O.project(O.rowmap(levels[0], maps[0]), zc), 0.5), F32_TOL, "full-width fused")


@pytest.mark.parametrize("small_max,chunk", [(4, 64), (8, 64), (32, 128), (1, 64)])
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_every_tier(oracle_mod, H, small_max, chunk, dtype):
    O = oracle_mod
    hg = tier_hypergraph(11, small_max, chunk)
    levels, maps, hier = both_hierarchies(O, H, hg, 1)
    d = 64
    opts = {"small_max": small_max, "chunk": chunk}
    plan = H.Plan(hier, d, dtype, options=opts)
    rng = np.random.default_rng(3)
    z0 = rng.standard_normal((levels[0].rows, d)).astype(np.float32)
    zin = z0 if dtype == "f32" else _bf16_round(z0)
    out = _host(plan.sweep(0, _dev(z0, dtype), 0.5))
    ref, E = oracle_sweep_bf16(O, levels[0], zin, None, 0.5)

    def check(got, what):
        if dtype == "f32":
            _assert_close(got, ref, F32_TOL, what)
        else:
            assert_bf16(got, ref, E, what)

    check(out, f"tiers {opts} {dtype}")
    # columns in two passes: a narrower lane group, so a different (fixed)
    # summation order; same tolerance, and repeatable bit for bit
    plan2 = H.Plan(hier, d, dtype, options=dict(opts, panel_cols=32))
    out2 = _host(plan2.sweep(0, _dev(z0, dtype), 0.5))
    check(out2, f"tiers {opts} {dtype} two panels")
    np.testing.assert_array_equal(_host(plan2.sweep(0, _dev(z0, dtype), 0.5)), out2)


# ---------------------------------------------------------------------------
# multi-level refinement
# ---------------------------------------------------------------------------

def _refine_case(O, H, cfg_name, dtype, cols=None, n_levels=None, sweeps=None):
    cfg = CONFIGS[cfg_name]
    hg = make_hypergraph(cfg)
    L = cfg.levels if n_levels is None else n_levels
    levels, maps, hier = both_hierarchies(O, H, hg, L)
    K = list(cfg.sweeps[: L + 1]) if sweeps is None else sweeps
    zc = coarsest_embedding(cfg, levels[-1].rows, cfg.d)
    plan = H.Plan(hier, cfg.d, dtype)
    zdev = _dev(zc, dtype)
    out, res, done = plan.refine(zdev, K, 0.5, residuals=True)
    got = _host(out)
    zin = zc if dtype == "f32" else _bf16_round(zc)
    c = slice(None) if cols is None else cols
    if dtype == "f32":
        ref, ref_res = O.refine(levels, maps, np.ascontiguousarray(zin[:, c]), K, 0.5, return_residuals=True)
        return got[:, c], ref, _host(res), np.array(ref_res), done, K
    # BF16: the refinement with the elementwise bound of its rounding error
    ref, E = oracle_refine_bf16(O, levels, maps, np.ascontiguousarray(zin[:, c]), K, 0.5)
    return got[:, c], ref, E, None, done, K


def test_refine_tiny2k_f32(oracle_mod, H):
    got, ref, res, ref_res, done, K = _refine_case(oracle_mod, H, "tiny-2k", "f32")
    _assert_close(got, ref, F32_TOL, "tiny-2k refine f32")
    assert list(done) == list(K)
    np.testing.assert_allclose(res[: len(ref_res)], ref_res, rtol=1e-5)


@pytest.mark.parametrize("sweeps", [[8, 9, 0, 17], [16, 1, 3, 0]])
def test_refine_residual_batches(oracle_mod, H, sweeps):
    """A fixed-count refinement reduces its residuals 8 sweeps of a level at
    a time: sweep counts that fill one or two batches exactly, leave a
    partial batch, or are 0 (a bare projection); every residual against the
    oracle's."""
    got, ref, res, ref_res, done, K = _refine_case(oracle_mod, H, "tiny-2k", "f32", sweeps=sweeps)
    _assert_close(got, ref, F32_TOL, f"tiny-2k refine {sweeps}")
    assert list(done) == list(K)
    assert len(ref_res) == sum(K)
    np.testing.assert_allclose(res[: len(ref_res)], ref_res, rtol=1e-5)


def test_refine_tiny2k_bf16(oracle_mod, H):
    got, ref, E, _, _, _ = _refine_case(oracle_mod, H, "tiny-2k", "bf16")
    assert_bf16(got, ref, E, "tiny-2k refine bf16")


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_refine_hub200k(oracle_mod, H, dtype):
    """Medium hub-heavy config, all columns."""
    got, ref, res, ref_res, _, _ = _refine_case(oracle_mod, H, "hub-200k", dtype)
    if dtype == "f32":
        _assert_close(got, ref, F32_TOL, "hub-200k refine f32")
    else:
        assert_bf16(got, ref, res, "hub-200k refine bf16")


@pytest.mark.parametrize("dtype", ["bf16", "f32"])
def test_refine_zipf2m_full_size_column_sample(oracle_mod, H, dtype):
    """The benchmark workload (2M nodes, 1.5M hyperedges, 8 coarsening
    steps, 20 sweeps per level, d = 128, default launch options) on the GPU;
    the oracle computes two of the 128 columns over every row (columns are
    independent under the sweep and the projection)."""
    cols = [0, 77]
    got, ref, res, ref_res, done, K = _refine_case(oracle_mod, H, "zipf-2m", dtype, cols=cols)
    if dtype == "f32":
        _assert_close(got, ref, F32_TOL, f"zipf-2m refine f32 cols {cols}")
    else:
        assert_bf16(got, ref, res, f"zipf-2m refine bf16 cols {cols}")


def test_refine_zero_and_tol(oracle_mod, H):
    """K = 0 levels (bare projections), omega = 0 (identity), early stop."""
    import torch
    O = oracle_mod
    hg = random_hypergraph(9, 400, 300, 2, 6, weighted=True)
    levels, maps, hier = both_hierarchies(O, H, hg, 3)
    d = 16
    plan = H.Plan(hier, d, "f32")
    zc = np.random.default_rng(0).standard_normal((levels[-1].rows, d)).astype(np.float32)
    for K in ([0, 0, 0, 0], [0, 3, 0, 2], [4, 0, 0, 0], [1, 1, 1, 1]):
        out, _, _ = plan.refine(_dev(zc), K, 0.5)
        _assert_close(_host(out), O.refine(levels, maps, zc, K, 0.5), F32_TOL, f"K={K}")
    out, _, _ = plan.refine(_dev(zc), [2, 2, 2, 2], 0.0)
    np.testing.assert_array_equal(_host(out), O.refine(levels, maps, zc, [0, 0, 0, 0], 0.5))
    # early stop (the epsilon rule of Section 4): the sweeps run per level and
    # every residual against the oracle's, for tol values that make levels
    # stop at different sweeps; each tol is kept clear of the oracle's
    # residuals so that FP32 rounding cannot flip a decision
    K = [50, 50, 50, 50]
    _, free_res = O.refine(levels, maps, zc, K, 0.5, return_residuals=True)
    for q in (0.2, 0.5, 0.8):
        tol = float(np.quantile(free_res, q))
        while True:
            ref, ref_res, ref_cnt = O.refine(levels, maps, zc, K, 0.5, tol=tol, return_residuals=True,
                                             return_counts=True)
            if min(abs(r - tol) for r in ref_res) > 1e-3 * tol:
                break
            tol *= 1.01
        out, res, done = plan.refine(_dev(zc), K, 0.5, tol=tol, residuals=True)
        assert list(done) == list(ref_cnt), (tol, list(done), ref_cnt)
        # a residual is the norm of a difference of two FP32-stored iterates:
        # relative 1e-5, and an absolute floor of a few FP32 roundings of Z
        np.testing.assert_allclose(_host(res)[: len(ref_res)], ref_res, rtol=1e-5,
                                   atol=4 * 2.0 ** -24 * float(np.linalg.norm(ref)))
        _assert_close(_host(out), ref, F32_TOL, f"tol={tol:.4g}")
    torch.cuda.synchronize()


def _hg(n_nodes, members, w=None):
    ptr = np.concatenate([[0], np.cumsum([len(m) for m in members])]).astype(np.int64)
    idx = np.array([v for m in members for v in m], dtype=np.int32)
    return n_nodes, len(members), ptr, idx, None if w is None else np.asarray(w, dtype=np.float32)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_degenerate_hypergraphs(oracle_mod, H, dtype):
    """Refinement and its reverse on degenerate inputs, against the oracle:
    nodes without any hyperedge (every row a fixed point, a coarsening
    step changes nothing), one hyperedge holding every node (the coarse
    level is one node and no hyperedge), hyperedges of one member, the
    narrowest width (d = 8) and omega = 1."""
    import torch
    O = oracle_mod
    tol = F32_TOL if dtype == "f32" else BF16_TOL
    rng = np.random.default_rng(41)
    cases = {
        "nodes only": _hg(7, []),
        "one hyperedge with every node": _hg(300, [list(range(300))]),
        "one-member hyperedges": _hg(50, [[v] for v in range(0, 50, 2)] + [[1, 3, 5], [7]], rng.uniform(0.5, 2, 27)),
    }
    for name, (n, m, ptr, idx, w) in cases.items():
        levels, maps = O.build_hierarchy(n, m, ptr, idx, w, 2)
        hier = H.Hierarchy.build(n, m, ptr, idx, w, 2)
        for d, omega in ((8, 0.5), (16, 1.0)):
            plan = H.Plan(hier, d, dtype)
            zc = rng.standard_normal((levels[-1].rows, d)).astype(np.float32)
            zr = zc if dtype == "f32" else _bf16_round(zc)
            out, _, _ = plan.refine(_dev(zc, dtype), [2, 3, 1], omega)
            if dtype == "f32":
                _assert_close(_host(out), O.refine(levels, maps, zr, [2, 3, 1], omega), tol,
                              f"{name} d={d} omega={omega}")
            else:
                ref, E = oracle_refine_bf16(O, levels, maps, zr, [2, 3, 1], omega)
                assert_bf16(_host(out), ref, E, f"{name} d={d} omega={omega}")
            if dtype == "f32" and omega > 0:
                y = rng.standard_normal((levels[0].rows, d)).astype(np.float32)
                g = rng.standard_normal((levels[0].rows, d)).astype(np.float32)
                z = plan.sweep(0, _dev(y), omega)
                dw = torch.zeros(max(levels[0].n_edges, 1), dtype=torch.float32, device="cuda")
                gy = plan.sweep_adjoint(0, _dev(g), _dev(y), z, omega, dw=dw)
                ref_gy, ref_dw = O.sweep_vjp(levels[0], y, g, omega)
                _assert_close(_host(gy), ref_gy, F32_TOL, f"{name} reverse")
                if levels[0].n_edges:
                    got = dw.cpu().numpy()[: levels[0].n_edges].astype(np.float64)
                    assert np.max(np.abs(got - ref_dw)) <= 1e-4 * max(1.0, np.max(np.abs(ref_dw))), name
    torch.cuda.synchronize()


def test_determinism_bitwise(oracle_mod, H):
    O = oracle_mod
    hg = tier_hypergraph(5, 8, 64)
    levels, maps, hier = both_hierarchies(O, H, hg, 2)
    plan = H.Plan(hier, 32, "bf16", options={"small_max": 8, "chunk": 64})
    zc = _dev(np.random.default_rng(1).standard_normal((levels[-1].rows, 32)), "bf16")
    a, ra, _ = plan.refine(zc, [3, 3, 3], 0.5, residuals=True)
    b, rb, _ = plan.refine(zc, [3, 3, 3], 0.5, residuals=True)
    import torch
    assert torch.equal(a.view(torch.int16), b.view(torch.int16))
    assert torch.equal(ra, rb)


def test_cast_round_to_nearest_even(H):
    import torch
    x = np.random.default_rng(0).standard_normal(10_000).astype(np.float32) * 100
    x[:4] = [1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -0.0, 3.0e38]   # exact ties and extremes
    t = H.cast(_dev(x), "bf16")
    ref = torch.as_tensor(x).to(torch.bfloat16)
    assert bool((t.cpu().view(torch.int16) == ref.view(torch.int16)).all())
    back = H.cast(t, "f32")
    assert bool((back.cpu() == ref.float()).all())


# ---------------------------------------------------------------------------
# reverse mode
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed,small_max,chunk,d", [(0, 32, 512, 32), (1, 4, 64, 64), (2, 1, 64, 16),
                                                     (3, 8, 128, 128)])
def test_sweep_adjoint(oracle_mod, H, seed, small_max, chunk, d):
    import torch
    O = oracle_mod
    hg = tier_hypergraph(seed, max(small_max, 2), chunk) if seed % 2 else \
        random_hypergraph(seed, 800, 500, 1, 10, weighted=True)
    levels, maps, hier = both_hierarchies(O, H, hg, 1)
    plan = H.Plan(hier, d, "f32", options={"small_max": small_max, "chunk": chunk})
    rng = np.random.default_rng(seed)
    theta = rng.uniform(-0.5, 0.5, size=levels[0].n_edges).astype(np.float32)
    wt = torch.empty(levels[0].n_edges, dtype=torch.float32, device="cuda")
    plan.set_edge_logweights(0, _dev(theta), w_out=wt)
    w_host = wt.cpu().numpy()
    y = rng.standard_normal((levels[0].rows, d)).astype(np.float32)
    g = rng.standard_normal((levels[0].rows, d)).astype(np.float32)
    omega = 0.5
    z = plan.sweep(0, _dev(y), omega)
    _assert_close(_host(z), O.sweep(levels[0], y, omega, 0, w_host), F32_TOL, "weighted forward")
    dw = torch.zeros(levels[0].n_edges, dtype=torch.float32, device="cuda")
    gy = plan.sweep_adjoint(0, _dev(g), _dev(y), z, omega, dw=dw)
    ref_gy, ref_dw = O.sweep_vjp(levels[0], y, g, omega, w_host)
    _assert_close(_host(gy), ref_gy, F32_TOL, "adjoint gy")
    _assert_close(dw.cpu().numpy(), ref_dw, GRAD_TOL, "adjoint dw")
    # project adjoint
    gc = plan.project_adjoint(0, _dev(g))
    _assert_close(_host(gc), O.project_vjp(O.rowmap(levels[0], maps[0]), levels[1].rows, g), F32_TOL,
                  "project adjoint")
    dth = plan.logweight_grad(0, dw.clone())
    _assert_close(dth.cpu().numpy(), ref_dw * w_host, GRAD_TOL, "dtheta")


@pytest.mark.parametrize("dtype,small_max,chunk,omega", [("f32", 32, 512, 0.5), ("f32", 4, 64, 0.3),
                                                          ("bf16", 8, 128, 0.5), ("bf16", 8, 128, 0.3),
                                                          ("bf16", 64, 512, 0.2)])
def test_split_weight_gradient(oracle_mod, H, dtype, small_max, chunk, omega):
    """K reverse sweeps with the weight gradient split (per-node part summed
    over the sweeps, gathered per hyperedge once by hnv_weight_grad_finish)
    against the gradient completed in every sweep and against the oracle;
    the cotangents are the same bit for bit with the gradient split, whole
    or not requested (without it the sweep reads neither y nor z)."""
    import torch
    O = oracle_mod
    hg = random_hypergraph(21, 3000, 2000, 1, 40, weighted=True)
    levels, maps, hier = both_hierarchies(O, H, hg, 1)
    d, K = 32, 3
    plan = H.Plan(hier, d, dtype, options={"small_max": small_max, "chunk": chunk})
    rng = np.random.default_rng(21)
    theta = rng.uniform(-0.5, 0.5, size=levels[0].n_edges).astype(np.float32)
    wt = torch.empty(levels[0].n_edges, dtype=torch.float32, device="cuda")
    plan.set_edge_logweights(0, _dev(theta), w_out=wt)
    w_host = wt.cpu().numpy()
    y0 = rng.standard_normal((levels[0].rows, d)).astype(np.float32)
    g0 = rng.standard_normal((levels[0].rows, d)).astype(np.float32)
    states = [_dev(y0, dtype)]
    for _ in range(K):
        states.append(plan.sweep(0, states[-1], omega))
    n_nodes, n_edges, _ = plan.level_info(0)

    def backward(mode):
        dw = torch.zeros(n_edges, dtype=torch.float32, device="cuda") if mode else None
        nacc = torch.zeros(n_nodes, dtype=torch.float32, device="cuda") if mode == "split" else None
        g = _dev(g0, dtype)
        for i in range(K, 0, -1):
            g = plan.sweep_adjoint(0, g, states[i - 1], states[i], omega, dw=dw, node_acc=nacc)
        if mode == "split":
            plan.weight_grad_finish(0, nacc, dw)
        return g, dw

    g_split, dw_split = backward("split")
    g_whole, dw_whole = backward("whole")
    g_none, _ = backward(None)
    assert torch.equal(g_split, g_whole) and torch.equal(g_split, g_none)
    assert rel_fro(dw_split.cpu().numpy(), dw_whole.cpu().numpy().astype(np.float64)) <= 1e-5
    # the oracle on the same (stored) forward states
    ref_dw = np.zeros(n_edges)
    gtop = _host(_dev(g0, dtype))
    gr = gtop
    for i in range(K, 0, -1):
        gr, dwi = O.sweep_vjp(levels[0], _host(states[i - 1]), gr, omega, w_host)
        ref_dw += dwi
    if dtype == "f32":
        _assert_close(_host(g_split), gr, F32_TOL, "split g f32")
        _assert_close(dw_split.cpu().numpy(), ref_dw, GRAD_TOL, "split dw f32")
    else:
        # BF16: the stored cotangents and the stored sweep outputs (from which
        # the node term's neighbour mean is recovered) round at 2^-8
        _assert_bf16_reverse(O, levels[0], [_host(t) for t in states[:K]], [_host(t) for t in states[1:]], gtop,
                             omega, w_host, 0, _host(g_split), gr, dw_split.cpu().numpy(), ref_dw,
                             f"split omega={omega}")


def test_refine_function_grad500k_shape_small(oracle_mod, H):
    """Differentiable refinement (projection + 10 sweeps with learnable
    log-weights, checkpoint every 5) on a reduced instance of the
    differentiable-refinement workload; loss = CE of a linear head."""
    import torch
    O = oracle_mod
    hg = random_hypergraph(4, 5000, 3000, 2, 20, weighted=False)
    levels, maps, hier = both_hierarchies(O, H, hg, 1)
    d, K = 32, 10
    plan = H.Plan(hier, d, "f32")
    rng = np.random.default_rng(4)
    zc = rng.standard_normal((levels[1].rows, d)).astype(np.float32)
    theta = rng.uniform(-0.3, 0.3, size=levels[0].n_edges).astype(np.float32)
    lab_nodes = np.sort(rng.choice(levels[0].n_nodes, size=500, replace=False))
    labels = rng.integers(0, 16, size=500)
    W = (rng.standard_normal((16, d)) / np.sqrt(d)).astype(np.float32)
    zc_t = _dev(zc).requires_grad_(True)
    th_t = _dev(theta).requires_grad_(True)
    out = H.refine_level(zc_t, th_t, plan, 0, K, 0.5, from_coarse=True, ckpt_every=5)
    logits = out[torch.as_tensor(lab_nodes).cuda()] @ _dev(W).t()
    loss = torch.nn.functional.cross_entropy(logits, torch.as_tensor(labels).cuda())
    loss.backward()
    w_dev = torch.as_tensor(theta).cuda().exp().cpu().numpy()
    zK, _, _ = O.finest_refine_vjp(levels[0], maps[0], zc, w_dev, K, 0.5, np.zeros((levels[0].rows, d)))
    ref_loss, dz_nodes = O.ce_head(zK[lab_nodes], labels, W, np.zeros(16))
    gK = np.zeros((levels[0].rows, d))
    gK[lab_nodes] = dz_nodes
    _, ref_gc, ref_dw = O.finest_refine_vjp(levels[0], maps[0], zc, w_dev, K, 0.5, gK)
    assert abs(loss.item() - ref_loss) <= 1e-5 * abs(ref_loss)
    _assert_close(_host(zc_t.grad), ref_gc, GRAD_TOL, "dL/dZc")
    _assert_close(th_t.grad.cpu().numpy(), ref_dw * w_dev, GRAD_TOL, "dL/dtheta")


@pytest.mark.parametrize("order", ["jacobi", "edge_first"])
def test_gradients_through_every_level(oracle_mod, H, order):
    """Reverse mode across the whole hierarchy: K sweeps at the coarsest
    level, then projection and K sweeps at each finer level, every level
    with learnable log-weights of its own; loss = <G, node rows of Z_0>.
    The gradients of the coarsest embedding and of every level's
    log-weights against the oracle's FP64 reverse pass composed level by
    level (the projection adjoint at every level boundary)."""
    import torch
    O = oracle_mod
    hg = random_hypergraph(14, 3000, 2000, 2, 10, weighted=True)
    levels, maps, hier = both_hierarchies(O, H, hg, 3)
    L = len(levels) - 1
    d, K, omega = 16, 4, 0.5
    plan = H.Plan(hier, d, "f32", options={"order": order})
    o = 1 if order == "edge_first" else 0
    rng = np.random.default_rng(14)
    zc = rng.standard_normal((levels[L].rows, d)).astype(np.float32)
    thetas = [rng.uniform(-0.5, 0.5, size=lv.n_edges).astype(np.float32) for lv in levels]
    G = rng.standard_normal((levels[0].n_nodes, d))
    zc_t = _dev(zc).requires_grad_(True)
    th_t = [_dev(t).requires_grad_(True) for t in thetas]
    z = H.refine_hierarchy(zc_t, th_t, plan, [K] * (L + 1), omega, ckpt_every=3)
    loss = (z[: levels[0].n_nodes] * _dev(G)).sum()
    loss.backward()

    ws = [np.exp(t.astype(np.float64)).astype(np.float32) for t in thetas]
    states = [zc.astype(np.float64)]
    for _ in range(K):
        states.append(O.sweep(levels[L], states[-1], omega, o, ws[L]))
    zs = {L: states[-1]}
    for l in range(L - 1, -1, -1):
        zs[l] = O.finest_refine_vjp(levels[l], maps[l], zs[l + 1], ws[l], K, omega,
                                    np.zeros((levels[l].rows, d)), o)[0]
    g = np.zeros((levels[0].rows, d))
    g[: levels[0].n_nodes] = G
    dws = {}
    for l in range(L):
        _, g, dws[l] = O.finest_refine_vjp(levels[l], maps[l], zs[l + 1], ws[l], K, omega, g, o)
    dws[L] = np.zeros(levels[L].n_edges)
    for i in range(K, 0, -1):
        g, dwi = O.sweep_vjp(levels[L], states[i - 1], g, omega, ws[L], o)
        dws[L] += dwi
    ref_loss = float((zs[0][: levels[0].n_nodes] * G).sum())
    assert abs(loss.item() - ref_loss) <= 1e-5 * np.abs(zs[0][: levels[0].n_nodes] * G).sum()
    _assert_close(_host(zc_t.grad), g, GRAD_TOL, "dL/dZ at the coarsest level")
    for l in range(L + 1):
        _assert_close(th_t[l].grad.cpu().numpy(), dws[l] * ws[l], GRAD_TOL, f"dL/dtheta at level {l}")


# ---------------------------------------------------------------------------
# full-size instances of the large workloads
# ---------------------------------------------------------------------------

def test_zipf8m_two_levels_forward_and_reverse(oracle_mod, H):
    """Friendster-scale hypergraph (8M nodes, 10M hyperedges, 125.5M
    incidences), BF16 storage: the full-size finest level and its first
    coarsening, 4 sweeps per level (the finest level's first one fused with
    the projection), then 3 reverse sweeps at the finest level.  The oracle
    computes two of the 128 columns; the reverse pass uses a cotangent that
    is zero outside those columns, so the hyperedge-weight gradient (a sum
    over columns) is exactly the two-column one."""
    import torch
    O = oracle_mod
    cfg = CONFIGS["zipf-8m"]
    hg = make_hypergraph(cfg)
    levels, maps, hier = both_hierarchies(O, H, hg, 1)
    cols = [5, 101]
    d = cfg.d
    plan = H.Plan(hier, d, "bf16")
    zc = coarsest_embedding(cfg, levels[1].rows, d, columns=cols)
    zfull = torch.zeros((levels[1].rows, d), dtype=torch.bfloat16, device="cuda")
    zfull[:, cols] = _dev(zc, "bf16")
    zin = _bf16_round(zc)
    K = [4, 4]
    out, _, _ = plan.refine(zfull, K, 0.5)
    ref, E = oracle_refine_bf16(O, levels, maps, zin, K, 0.5)
    assert_bf16(_host(out[:, cols].contiguous()), ref, E, "zipf-8m forward")
    # reverse: 3 sweeps at level 0 from the refined state, seeded cotangent on two columns
    y0 = out
    states = [y0]
    for _ in range(3):
        states.append(plan.sweep(0, states[-1], 0.5))
    gsmall = np.random.default_rng(305).standard_normal((levels[0].rows, 2)).astype(np.float32)
    gd = torch.zeros((levels[0].rows, d), dtype=torch.bfloat16, device="cuda")
    gd[:, cols] = _dev(gsmall, "bf16")
    dw = torch.zeros(levels[0].n_edges, dtype=torch.float32, device="cuda")
    for i in range(3, 0, -1):
        gd = plan.sweep_adjoint(0, gd, states[i - 1], states[i], 0.5, dw=dw)
    # the oracle's reverse pass on the same two columns of the stored forward
    # states, held to the BF16 reverse-mode bound
    ys = [_host(t[:, cols].contiguous()) for t in states]
    go = _bf16_round(gsmall)
    gtop = go
    dwo = np.zeros(levels[0].n_edges)
    for i in range(3, 0, -1):
        go, dwi = O.sweep_vjp(levels[0], ys[i - 1], go, 0.5)
        dwo += dwi
    _assert_bf16_reverse(O, levels[0], ys[:3], ys[1:], gtop, 0.5, None, 0, _host(gd[:, cols].contiguous()), go,
                         dw.cpu().numpy(), dwo, "zipf-8m reverse")
    other = torch.as_tensor([c for c in range(d) if c not in cols], device="cuda")
    assert float(gd.index_select(1, other).abs().max().float().item()) == 0.0


def test_grad500k_full_size_gradients(oracle_mod, H):
    """Differentiable refinement at full size (500K nodes, 300K hyperedges,
    d = 128 FP32): projection + 10 sweeps with learnable log-weights,
    checkpoint every 5, CE head on 10% of the nodes with seeded labels."""
    import torch
    from synth import labelled_nodes, linear_head
    O = oracle_mod
    cfg = CONFIGS["grad-500k"]
    hg = make_hypergraph(cfg)
    levels, maps, hier = both_hierarchies(O, H, hg, cfg.levels)
    plan = H.Plan(hier, cfg.d, "f32")
    K = cfg.sweeps[0]
    zc = coarsest_embedding(cfg, levels[1].rows, cfg.d)
    theta = (np.random.default_rng(304).uniform(-0.3, 0.3, size=hg.n_edges)).astype(np.float32)
    nodes, labels = labelled_nodes(cfg)
    W, b = linear_head(cfg)
    zc_t = _dev(zc).requires_grad_(True)
    th_t = _dev(theta).requires_grad_(True)
    out = H.refine_level(zc_t, th_t, plan, 0, K, 0.5, from_coarse=True, ckpt_every=cfg.checkpoint_every)
    logits = out[torch.as_tensor(nodes).cuda()] @ _dev(W).t() + _dev(b)
    loss = torch.nn.functional.cross_entropy(logits, torch.as_tensor(labels).cuda())
    loss.backward()
    w = torch.as_tensor(theta).cuda().exp().cpu().numpy()
    zK, _, _ = O.finest_refine_vjp(levels[0], maps[0], zc, w, K, 0.5, np.zeros((levels[0].rows, cfg.d)))
    ref_loss, dz_nodes = O.ce_head(zK[nodes], labels, W, b)
    gK = np.zeros((levels[0].rows, cfg.d))
    gK[nodes] = dz_nodes
    _, ref_gc, ref_dw = O.finest_refine_vjp(levels[0], maps[0], zc, w, K, 0.5, gK)
    assert abs(loss.item() - ref_loss) <= 1e-5 * abs(ref_loss)
    _assert_close(_host(zc_t.grad), ref_gc, GRAD_TOL, "grad-500k dL/dZc")
    _assert_close(th_t.grad.cpu().numpy(), ref_dw * w, GRAD_TOL, "grad-500k dL/dtheta")


# ---------------------------------------------------------------------------
# edge-first order (hyperedge rows first, then node rows from the new ones)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("small_max,chunk", [(64, 512), (4, 64)])
def test_edge_first_sweeps(oracle_mod, H, dtype, small_max, chunk):
    import torch
    O = oracle_mod
    hg = tier_hypergraph(7, max(small_max, 2), chunk)
    levels, maps, hier = both_hierarchies(O, H, hg, 2)
    d = 64
    plan = H.Plan(hier, d, dtype, options={"order": "edge_first", "small_max": small_max, "chunk": chunk})
    tol = F32_TOL if dtype == "f32" else BF16_TOL
    rng = np.random.default_rng(8)
    z0 = rng.standard_normal((levels[0].rows, d)).astype(np.float32)
    zc = rng.standard_normal((levels[1].rows, d)).astype(np.float32)
    z0r = z0 if dtype == "f32" else _bf16_round(z0)
    zcr = zc if dtype == "f32" else _bf16_round(zc)
    resid = torch.zeros(1, dtype=torch.float64, device="cuda")
    ref, E = oracle_sweep_bf16(O, levels[0], z0r, None, 0.5, 1)

    def check(got, want, bound, what):
        if dtype == "f32":
            _assert_close(got, want, F32_TOL, what)
        else:
            assert_bf16(got, want, bound, what)

    check(_host(plan.sweep(0, _dev(z0, dtype), 0.5, resid=resid)), ref, E, "edge-first sweep")
    assert abs(resid.item() - O.residual(ref, z0r)) <= 10 * tol * O.residual(ref, z0r)
    # in place
    zi = _dev(z0, dtype)
    plan.sweep(0, zi, 0.5, out=zi)
    check(_host(zi), ref, E, "edge-first in place")
    # fused with the projection
    ref_f, E_f = oracle_sweep_bf16(O, levels[0], O.project(O.rowmap(levels[0], maps[0]), zcr), None, 0.5, 1)
    check(_host(plan.sweep(0, _dev(zc, dtype), 0.5, from_coarse=True)), ref_f, E_f, "edge-first fused")
    # multi-level
    ztop = rng.standard_normal((levels[2].rows, d)).astype(np.float32)
    ztr = ztop if dtype == "f32" else _bf16_round(ztop)
    out, _, _ = plan.refine(_dev(ztop, dtype), [3, 2, 4], 0.5)
    ref_r, E_r = oracle_refine_bf16(O, levels, maps, ztr, [3, 2, 4], 0.5, order=1)
    check(_host(out), ref_r, E_r, "edge-first refine")


@pytest.mark.parametrize("dtype,small_max,chunk,d", [("f32", 32, 512, 32), ("f32", 4, 64, 64), ("bf16", 8, 128, 128),
                                                     ("bf16", 1, 64, 16)])
def test_edge_first_adjoint(oracle_mod, H, dtype, small_max, chunk, d):
    """Reverse mode of the edge-first order: one reverse sweep (cotangent and
    the hyperedge-weight gradient) against the oracle's, then K reverse
    sweeps with the weight gradient whole, split and not requested: the
    cotangents are the same bit for bit, the split gradient matches the
    whole one and the oracle's."""
    import torch
    O = oracle_mod
    hg = tier_hypergraph(31, max(small_max, 2), chunk) if small_max < 32 else \
        random_hypergraph(31, 2000, 1200, 1, 12, weighted=True)
    levels, maps, hier = both_hierarchies(O, H, hg, 1)
    plan = H.Plan(hier, d, dtype, options={"order": "edge_first", "small_max": small_max, "chunk": chunk})
    tol = F32_TOL if dtype == "f32" else BF16_TOL
    rng = np.random.default_rng(31)
    theta = rng.uniform(-0.5, 0.5, size=levels[0].n_edges).astype(np.float32)
    wt = torch.empty(levels[0].n_edges, dtype=torch.float32, device="cuda")
    plan.set_edge_logweights(0, _dev(theta), w_out=wt)
    w_host = wt.cpu().numpy()
    omega, K = 0.6, 3
    y0 = rng.standard_normal((levels[0].rows, d)).astype(np.float32)
    g0 = rng.standard_normal((levels[0].rows, d)).astype(np.float32)
    states = [_dev(y0, dtype)]
    for _ in range(K):
        states.append(plan.sweep(0, states[-1], omega))
    if dtype == "f32":
        _assert_close(_host(states[1]), O.sweep(levels[0], _host(states[0]), omega, 1, w_host), tol, "forward")
    else:
        ref1, E1 = oracle_sweep_bf16(O, levels[0], _host(states[0]), None, omega, 1, w_host)
        assert_bf16(_host(states[1]), ref1, E1, "forward")
    n_nodes, n_edges, _ = plan.level_info(0)
    # one reverse sweep
    dw1 = torch.zeros(n_edges, dtype=torch.float32, device="cuda")
    g1 = plan.sweep_adjoint(0, _dev(g0, dtype), states[0], states[1], omega, dw=dw1)
    gtop = _host(_dev(g0, dtype))
    ref_g1, ref_dw1 = O.sweep_vjp(levels[0], _host(states[0]), gtop, omega, w_host, order=1)
    if dtype == "f32":
        _assert_close(_host(g1), ref_g1, F32_TOL, "edge-first adjoint g")
        _assert_close(dw1.cpu().numpy(), ref_dw1, GRAD_TOL, "edge-first adjoint dw")
    else:
        _assert_bf16_reverse(O, levels[0], [_host(states[0])], [_host(states[1])], gtop, omega, w_host, 1,
                             _host(g1), ref_g1, dw1.cpu().numpy(), ref_dw1, "edge-first one sweep")

    def backward(mode):
        dw = torch.zeros(n_edges, dtype=torch.float32, device="cuda") if mode else None
        nacc = torch.zeros(n_nodes, dtype=torch.float32, device="cuda") if mode == "split" else None
        g = _dev(g0, dtype)
        for i in range(K, 0, -1):
            g = plan.sweep_adjoint(0, g, states[i - 1], states[i], omega, dw=dw, node_acc=nacc)
        if mode == "split":
            plan.weight_grad_finish(0, nacc, dw)
        return g, dw

    g_split, dw_split = backward("split")
    g_whole, dw_whole = backward("whole")
    g_none, _ = backward(None)
    assert torch.equal(g_split, g_whole) and torch.equal(g_split, g_none)
    assert rel_fro(dw_split.cpu().numpy(), dw_whole.cpu().numpy().astype(np.float64)) <= 1e-5
    ref_dw = np.zeros(n_edges)
    gr = gtop
    for i in range(K, 0, -1):
        gr, dwi = O.sweep_vjp(levels[0], _host(states[i - 1]), gr, omega, w_host, order=1)
        ref_dw += dwi
    if dtype == "f32":
        _assert_close(_host(g_split), gr, F32_TOL, "edge-first K reverse sweeps g")
        _assert_close(dw_split.cpu().numpy(), ref_dw, GRAD_TOL, "edge-first K reverse sweeps dw")
    else:
        _assert_bf16_reverse(O, levels[0], [_host(t) for t in states[:K]], [_host(t) for t in states[1:]], gtop,
                             omega, w_host, 1, _host(g_split), gr, dw_split.cpu().numpy(), ref_dw,
                             "edge-first K reverse sweeps")


# ---------------------------------------------------------------------------
# hyperedge-prediction features
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dtype,d", [("f32", 128), ("bf16", 128), ("f32", 24), ("bf16", 64), ("f32", 512)])
@pytest.mark.parametrize("op", ["variance", "mean", "min", "max"])
def test_score_candidates(oracle_mod, H, dtype, d, op):
    import torch
    O = oracle_mod
    rng = np.random.default_rng(d)
    n_nodes = 3000
    sizes = list(rng.integers(1, 12, size=400)) + [0, 600, 1500, 70, 64, 65, 512, 513, 2]
    sets = [sorted(rng.choice(n_nodes, size=k, replace=False).tolist()) for k in sizes]
    ptr = np.concatenate([[0], np.cumsum([len(s) for s in sets])]).astype(np.int64)
    idx = np.array([v for s in sets for v in s], dtype=np.int32)
    z = rng.standard_normal((n_nodes, d)).astype(np.float32) * 3 + 1
    zin = z if dtype == "f32" else _bf16_round(z)
    plan = H.ScorePlan(ptr, idx, n_nodes, d, dtype)
    got = plan.score(_dev(z, dtype), op).cpu().numpy()
    ref = O.score_candidates(zin, ptr, idx, op)
    # repeatable bit for bit
    np.testing.assert_array_equal(plan.score(_dev(z, dtype), op).cpu().numpy(), got)
    # a member outside the matrix is rejected when planning
    from paper_2103_09660_amd._lib import HNV_ERANGE, HnvError
    bad = idx.copy()
    bad[7] = n_nodes
    with pytest.raises(HnvError) as ei:
        H.ScorePlan(ptr, bad, n_nodes, d, dtype)
    assert ei.value.status == HNV_ERANGE
    assert np.array_equal(np.isnan(got), np.isnan(ref))
    ok = ~np.isnan(ref[:, 0])
    if op in ("min", "max"):
        np.testing.assert_array_equal(got[ok], ref[ok])
    else:
        _assert_close(got[ok], ref[ok], F32_TOL, f"score {op} {dtype} d={d}")
