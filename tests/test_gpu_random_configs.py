"""Randomised parity sweep: seeded random shapes, widths, storage types,
tier bounds, update orders and plan builders, each refined over a small
hierarchy on the GPU and compared with the FP64 oracle run on the same
(storage-rounded) input.  Every case is reproducible from its seed."""
import numpy as np
import pytest

from tests.cases import assert_bf16, assert_close, oracle_refine_bf16, random_hypergraph

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2103_09660_amd as H
    return H


def _case(seed):
    rng = np.random.default_rng(10_000 + seed)
    n_nodes = int(rng.integers(1, 4000))
    n_edges = int(rng.integers(1, 3000))
    hi = int(rng.choice([2, 4, 9, 30, 120]))
    d = int(8 * rng.integers(1, 65))
    dtype = str(rng.choice(["f32", "bf16"]))
    small_max = int(rng.choice([0, 1, 3, 8, 17, 64]))
    chunk = int(rng.choice([0, 5, 32, 100, 512]))
    order = str(rng.choice(["jacobi", "edge_first"]))
    weighted = bool(rng.integers(0, 2))
    levels = int(rng.integers(0, 4))
    sweeps = [int(k) for k in rng.integers(0, 4, size=levels + 1)]
    omega = float(rng.choice([0.25, 0.5, 0.9, 1.0]))
    build = str(rng.choice(["host", "device"]))
    return dict(n_nodes=n_nodes, n_edges=n_edges, hi=hi, d=d, dtype=dtype, small_max=small_max, chunk=chunk,
                order=order, weighted=weighted, levels=levels, sweeps=sweeps, omega=omega, build=build)


@pytest.mark.parametrize("seed", range(100))
def test_random_configuration(oracle_mod, H, seed):
    import torch
    O = oracle_mod
    c = _case(seed)
    print("case", seed, c, flush=True)
    hg = random_hypergraph(seed, c["n_nodes"], c["n_edges"], 1, c["hi"], weighted=c["weighted"])
    levels, maps = O.build_hierarchy(hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, hg.edge_w, c["levels"])
    hier = H.Hierarchy.build(hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, hg.edge_w, c["levels"])
    opts = {"small_max": c["small_max"], "chunk": c["chunk"], "order": c["order"]}
    plan = H.Plan(hier, c["d"], c["dtype"], options=opts, build=c["build"])
    rng = np.random.default_rng(seed)
    zc = rng.standard_normal((levels[-1].rows, c["d"])).astype(np.float32)
    zdev = torch.as_tensor(zc).cuda()
    if c["dtype"] == "bf16":
        zdev = zdev.to(torch.bfloat16)
        zin = zdev.float().cpu().numpy().astype(np.float64)
    else:
        zin = zc.astype(np.float64)
    out, _, done = plan.refine(zdev, c["sweeps"], c["omega"])
    got = out.float().cpu().numpy().astype(np.float64)
    order = 1 if c["order"] == "edge_first" else 0
    if c["dtype"] == "f32":
        ref = O.refine(levels, maps, zin, c["sweeps"], c["omega"], order=order)
    else:
        ref, E = oracle_refine_bf16(O, levels, maps, zin, c["sweeps"], c["omega"], order=order)
    assert list(done) == c["sweeps"]
    if np.linalg.norm(ref) == 0:
        assert np.abs(got).max() == 0
    elif c["dtype"] == "f32":
        assert_close(got, ref, 1e-5, f"case {seed} {c}")
    else:
        assert_bf16(got, ref, E, f"case {seed} {c}")


@pytest.mark.parametrize("seed", range(60))
def test_random_coarsening(oracle_mod, H, seed):
    """GPU coarsening, featureless and feature-driven, against the oracle bit
    for bit on seeded random shapes (integer weights force many key ties)."""
    import torch
    from synth import bag_of_words
    O = oracle_mod
    rng = np.random.default_rng(20_000 + seed)
    n_nodes = int(rng.integers(1, 3000))
    n_edges = int(rng.integers(1, 2500))
    hi = int(rng.choice([1, 2, 5, 20, 80]))
    weights = str(rng.choice(["none", "int", "float"]))
    k = int(4 * rng.integers(1, 40))
    print("case", seed, n_nodes, n_edges, hi, weights, k, flush=True)
    hg = random_hypergraph(seed, n_nodes, n_edges, 1, hi, weighted=weights != "none",
                           integer_weights=weights == "int")
    lv = O.Level(hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, hg.edge_w)
    dl = H.DeviceLevel.from_host(H.HostLevel(hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, hg.edge_w), "cuda")
    ref = O.coarsen_level(lv)
    nrep, erep, c = H.coarsen_level_device(dl)
    assert np.array_equal(nrep.cpu().numpy(), ref.node_rep) and np.array_equal(erep.cpu().numpy(), ref.edge_rep)
    assert np.array_equal(c.edge_ptr.cpu().numpy(), ref.coarse.eptr)
    assert np.array_equal(c.edge_idx.cpu().numpy(), ref.coarse.eidx)
    x = bag_of_words(30_000 + seed, n_nodes, k, 1, min(12, k), empty_frac=0.1, repeat_frac=0.3)
    fref, xref = O.coarsen_level_features(lv, x)
    fnrep, ferep, fc, xc = H.coarsen_level_features_device(dl, torch.as_tensor(x).cuda())
    assert np.array_equal(fnrep.cpu().numpy(), fref.node_rep) and np.array_equal(ferep.cpu().numpy(), fref.edge_rep)
    assert np.array_equal(fc.edge_idx.cpu().numpy(), fref.coarse.eidx)
    assert np.array_equal(xc.cpu().numpy(), xref)


@pytest.mark.parametrize("seed", range(40))
def test_random_reverse_mode(oracle_mod, H, seed):
    """Adjoint sweep, weight gradient and projection adjoint (FP32) against
    the oracle's reverse pass on seeded random shapes, widths, tier bounds,
    ω, hyperedge weights and sweep orders."""
    import torch
    O = oracle_mod
    rng = np.random.default_rng(40_000 + seed)
    n_nodes = int(rng.integers(2, 3000))
    n_edges = int(rng.integers(1, 2000))
    hi = int(rng.choice([2, 5, 20, 90]))
    d = int(8 * rng.integers(1, 33))
    small_max = int(rng.choice([0, 1, 4, 16]))
    chunk = int(rng.choice([0, 7, 64]))
    omega = float(rng.choice([0.3, 0.5, 1.0]))
    build = str(rng.choice(["host", "device"]))
    order = str(rng.choice(["jacobi", "edge_first"]))
    o = 1 if order == "edge_first" else 0
    print("case", seed, n_nodes, n_edges, hi, d, small_max, chunk, omega, build, order, flush=True)
    hg = random_hypergraph(seed, n_nodes, n_edges, 1, hi, weighted=True)
    levels, maps = O.build_hierarchy(hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, hg.edge_w, 1)
    hier = H.Hierarchy.build(hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, hg.edge_w, 1)
    plan = H.Plan(hier, d, "f32", options={"small_max": small_max, "chunk": chunk, "order": order}, build=build)
    w = hg.edge_w.astype(np.float32)
    y = rng.standard_normal((levels[0].rows, d)).astype(np.float32)
    g = rng.standard_normal((levels[0].rows, d)).astype(np.float32)
    yd, gd = torch.as_tensor(y).cuda(), torch.as_tensor(g).cuda()
    z = plan.sweep(0, yd, omega)
    dw = torch.zeros(levels[0].n_edges, dtype=torch.float32, device="cuda")
    gy = plan.sweep_adjoint(0, gd, yd, z, omega, dw=dw)
    ref_gy, ref_dw = O.sweep_vjp(levels[0], y, g, omega, w, o)
    assert_close(gy.cpu().numpy(), ref_gy, 1e-5, f"case {seed} dL/dy")
    # dw_e = ω Σ_{v∈e} <g_v, y_e - z~_v> / S_v (e'_e, the new hyperedge row, in
    # place of y_e in the edge-first order) can cancel to ~0 (a member with one
    # hyperedge has z~_v = y_e), and so can each dot product, so each entry is
    # held to 1e-4 of the sizes its rounding errors scale with: the products
    # |g_v|·|y_e| of the dot products (a floating-point dot product's error is
    # bounded by a multiple of sum_i |x_i y_i|) and, for z~_v = (z_v - (1-ω) y_v)/ω
    # recovered from the stored rows, |g_v|·(|z_v| + (1-ω)|y_v|)/ω
    lv0 = levels[0]
    z_ref = O.sweep(lv0, y, omega, o, w)
    nv = lv0.n_nodes
    S = np.zeros(nv)
    np.add.at(S, lv0.eidx, np.repeat(w.astype(np.float64), np.diff(lv0.eptr)))
    e_of = np.repeat(np.arange(lv0.n_edges), np.diff(lv0.eptr))
    ag = np.abs(g[lv0.eidx].astype(np.float64))
    ye = np.abs(y[nv + e_of].astype(np.float64) if o == 0 else z_ref[nv + e_of])
    rec = (np.abs(z_ref[:nv]) + (1 - omega) * np.abs(y[:nv].astype(np.float64))) / omega
    terms = (np.einsum("ij,ij->i", ag, ye) + np.einsum("ij,ij->i", ag, rec[lv0.eidx])) / S[lv0.eidx]
    scale = omega * np.bincount(e_of, weights=terms, minlength=lv0.n_edges)
    err = np.abs(dw.cpu().numpy().astype(np.float64) - ref_dw)
    assert np.all(err <= 1e-4 * scale + 1e-30), float(np.max(err / np.maximum(scale, 1e-30)))
    gc = plan.project_adjoint(0, gd)
    ref_gc = O.project_vjp(O.rowmap(levels[0], maps[0]), levels[1].rows, g)
    assert_close(gc.cpu().numpy(), ref_gc, 1e-5, f"case {seed} projection adjoint")
