"""Shared input builders for the parity tests: the same seeded hypergraph goes
to the oracle (its own hierarchy) and to the library (its own hierarchy);
the two hierarchies are compared bit for bit before any embedding is."""
import numpy as np

from synth import CONFIGS, coarsest_embedding, make_hypergraph, random_hypergraph


def rel_fro(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def max_abs_rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)) if b.size else 0.0


BF16_U = 2.0 ** -8   # unit roundoff of bfloat16 (8 significant bits), round to nearest even


F32_U = 2.0 ** -24   # unit roundoff of FP32


def _degrees(lv):
    """Neighbour count of every star-expansion row (nodes, then hyperedges)."""
    return np.concatenate([np.diff(lv.nptr), np.diff(lv.eptr)]).astype(np.float64)


def oracle_sweep_bf16(O, lv, z, E, omega, order=0, w=None):
    """One oracle sweep of z, and the elementwise first-order bound of the
    rounding error the same sweep accumulates when it runs in BF16 storage
    with FP32 arithmetic, given the bound E of its input's error:
      * the sweep matrix M (Jacobi, or the edge-first product of two
        relaxations) is non-negative and row-stochastic, so the input's
        error propagates elementwise as M applied to E;
      * every stored result rounds with |error| <= u |z'| (u = 2^-8);
      * the FP32 sum over a row's deg neighbours errs by at most about
        (deg + 3) 2^-24 (M |z|);
      * in the edge-first order the new hyperedge rows are stored before the
        node rows read them: their rounding enters node v with weight
        omega w_e / S_v.
    Returns (z', E')."""
    z_new = O.sweep(lv, z, omega, order, w)
    E_new = O.sweep(lv, E, omega, order, w) if E is not None else np.zeros_like(z_new)
    E_new += BF16_U * np.abs(z_new)
    E_new += (_degrees(lv)[:, None] + 3) * F32_U * O.sweep(lv, np.abs(z), omega, order, w)
    if order == 1 and lv.n_edges:
        from scipy.sparse import csr_matrix
        nv = lv.n_nodes
        wf = np.ones(lv.n_edges) if (w if w is not None else lv.w) is None else \
            np.asarray(w if w is not None else lv.w, dtype=np.float64)
        v_of = np.repeat(np.arange(nv), np.diff(lv.nptr))
        S = np.bincount(v_of, weights=wf[lv.nidx], minlength=nv)
        A = csr_matrix((wf[lv.nidx] / S[v_of], (v_of, lv.nidx)), shape=(nv, lv.n_edges))
        E_new[:nv] += omega * (A @ (BF16_U * np.abs(z_new[nv:])))
    return z_new, E_new


def oracle_refine_bf16(O, levels, maps, zin, sweeps, omega, order=0):
    """The oracle's multi-level refinement of zin (the BF16-rounded coarsest
    embedding, which both sides share, so the input carries no error) and
    the bound E of the BF16 run's rounding error, carried level to level
    by the projection (a copy) and sweep to sweep by oracle_sweep_bf16."""
    L = len(levels) - 1
    z = np.ascontiguousarray(zin, dtype=np.float64)
    E = np.zeros_like(z)
    for lvl in range(L, -1, -1):
        if lvl < L:
            rm = O.rowmap(levels[lvl], maps[lvl])
            z, E = O.project(rm, z), O.project(rm, E)
        for _ in range(int(sweeps[lvl])):
            z, E = oracle_sweep_bf16(O, levels[lvl], z, E, omega, order)
    return z, E


def assert_bf16(got, ref, E, what="", tol=1e-2):
    """BF16 parity: the Frobenius norm of the difference <= tol (1e-2) that
    of ref, and every element within twice its first-order rounding bound
    (second-order terms and slack) plus the FP32 tolerance."""
    ref = np.asarray(ref, dtype=np.float64)
    assert rel_fro(got, ref) <= tol, f"{what}: rel_fro={rel_fro(got, ref):.3e} > {tol}"
    assert_within(got, ref, 2 * np.asarray(E) + 1e-5 * (np.abs(ref) + np.sqrt(np.mean(ref * ref))), what)


def assert_close(got, ref, tol, what="", elem_tol=None):
    """Parity at a relative tolerance, element by element:
    |got_ij - ref_ij| <= t * (|ref_ij| + rms(ref)) for every entry, with
    t = elem_tol or tol (the rms term keeps entries that are near zero by
    cancellation from demanding a relative accuracy no storage format has),
    and the Frobenius norm of the difference <= tol * that of ref."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert got.shape == ref.shape, (what, got.shape, ref.shape)
    if ref.size == 0:
        return
    assert np.all(np.isfinite(got)), f"{what}: non-finite values"
    t = tol if elem_tol is None else elem_tol
    rms = float(np.sqrt(np.mean(ref * ref)))
    err = np.abs(got - ref)
    bound = t * (np.abs(ref) + rms)
    ratio = err / np.maximum(bound, 1e-300)
    worst = float(np.max(ratio))
    r = rel_fro(got, ref)
    assert worst <= 1.0 and r <= tol, (f"{what}: worst element at {worst:.3f} of its bound "
                                       f"(index {np.unravel_index(np.argmax(ratio), ratio.shape)}), "
                                       f"rel_fro={r:.3e}, tol={tol}, element tol={t}")


def assert_within(got, ref, bound, what=""):
    """|got - ref| <= bound element by element (a bound derived per entry)."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    err = np.abs(got - ref)
    ratio = err / np.maximum(bound, 1e-300)
    i = np.unravel_index(np.argmax(ratio), ratio.shape) if ratio.size else ()
    assert ratio.size == 0 or float(ratio[i]) <= 1.0, (
        f"{what}: worst element at {float(ratio[i]):.3f} of its bound (index {i}, error {float(err[i]):.3e}, "
        f"bound {float(np.asarray(bound)[i] if np.ndim(bound) else bound):.3e})")


def bf16_reverse_bounds(O, lv, ys, zs, g_top, omega, w=None, order=0):
    """Elementwise first-order bounds of the rounding error of K reverse
    sweeps run in BF16 storage (FP32 arithmetic), against the FP64 oracle run
    on the same stored forward states and the same BF16 cotangent.

    ys[i], zs[i]: input and output of forward sweep i (i = 0 .. K-1) as the
    GPU stored them (BF16 values, exact in FP64); g_top: the cotangent of the
    last output, BF16-rounded.  The reverse sweeps run from i = K-1 down to 0.

    Sources, with u = 2^-8:
      * the stored cotangent of every reverse sweep rounds with
        |error| <= u |g|; the reverse map has non-negative coefficients
        (1-omega, omega/|e|, omega w_e/S_v), so earlier errors propagate
        elementwise as the same map applied to their bounds;
      * the edge-first order also stores ge_e = dL/de'_e in BF16 before the
        node rows gather it: u |ge_e|, carried to node v with omega/|e|;
      * the node term of dL/dw_e needs zt_v, which the GPU recovers as
        (z_v - (1-omega) y_v)/omega from the stored z_v (the sweep's output
        rounded to BF16): |error of zt_v| <= u |z_v| / omega, and the factor
        omega of dL/dw cancels the 1/omega, leaving
        sum_{v in e} <|g_v|, u |z_v|> / S_v per hyperedge;
      * the cotangent's own error enters dL/dw_e through
        omega sum_{v in e} <E_v, |y_e| + |zt_v|> / S_v;
      * in the edge-first order the hyperedge term takes the stored new
        hyperedge row e'_e = z_e (|error| <= u |z_e|) in place of y_e.
    Returns (bound on the final cotangent, bound on dL/dw summed over the
    sweeps).  Callers add an FP32 floor (the arithmetic itself) on top."""
    from scipy.sparse import csr_matrix
    K = len(ys)
    nv, ne = lv.n_nodes, lv.n_edges
    wf = np.ones(ne) if w is None else np.asarray(w, dtype=np.float64)
    sizes = np.diff(lv.eptr)
    e_of = np.repeat(np.arange(ne), sizes)
    mem = lv.eidx.astype(np.int64)
    S = np.bincount(mem, weights=wf[e_of], minlength=nv)
    Sinv = np.where(S > 0, 1.0 / np.where(S > 0, S, 1.0), 0.0)
    A_S = csr_matrix((Sinv[mem], (e_of, mem)), shape=(ne, nv))           # hyperedge <- members / S_v
    A_E = csr_matrix((1.0 / sizes[e_of], (mem, e_of)), shape=(nv, ne))  # node <- hyperedges / |e|
    u = BF16_U

    def rowdot(a, b):
        return np.einsum("ij,ij->i", a, b)

    g = np.asarray(g_top, dtype=np.float64)
    E = np.zeros_like(g)
    B = np.zeros(ne)
    for i in range(K - 1, -1, -1):
        y = np.asarray(ys[i], dtype=np.float64)
        z = np.asarray(zs[i], dtype=np.float64)
        zt = (O.sweep(lv, y, omega, order, w) - (1 - omega) * y)[:nv] / omega
        he = np.abs(y[nv:]) if order == 0 else np.abs(z[nv:])
        aG, aE = np.abs(g[:nv]), E[:nv]
        t = omega * rowdot(A_S @ aE, he) + omega * (A_S @ rowdot(aE, np.abs(zt)))
        t += u * (A_S @ rowdot(aG + aE, np.abs(z[:nv])))
        if order == 1:
            t += omega * u * rowdot(A_S @ (aG + aE), np.abs(z[nv:]))
        B += t
        # the next cotangent: the exact one, and its error bound propagated
        # through the same (non-negative) reverse map plus this sweep's roundings
        g_next, _ = O.sweep_vjp(lv, y, g, omega, w, order)
        E_next, _ = O.sweep_vjp(lv, y, E, omega, w, order)
        E_next += u * np.abs(g_next)
        if order == 1:
            ge = g[nv:] + omega * wf[:, None] * (A_S @ g[:nv])
            E_next[:nv] += omega * u * (A_E @ np.abs(ge))
        g, E = g_next, E_next
    return E, B


def both_hierarchies(O, H, hg, n_coarsen):
    """(oracle levels, oracle maps, library Hierarchy), checked identical."""
    levels, maps = O.build_hierarchy(hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, hg.edge_w, n_coarsen)
    hier = H.Hierarchy.build(hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, hg.edge_w, n_coarsen)
    for a, b in zip(hier.levels, levels):
        assert a.n_nodes == b.n_nodes and a.n_edges == b.n_edges
        assert np.array_equal(a.edge_ptr, b.eptr) and np.array_equal(a.edge_idx, b.eidx)
    for a, b in zip(hier.maps, maps):
        assert np.array_equal(a.node_rep, b.node_rep) and np.array_equal(a.edge_rep, b.edge_rep)
    return levels, maps, hier


def tier_hypergraph(seed, small_max, chunk):
    """A hypergraph whose rows land on every tier boundary: hyperedges of
    size 1, small_max, small_max + 1, chunk, chunk + 1, several chunks, and
    nodes of degree 0, 1, small_max, small_max + 1, chunk + 1 and a hub."""
    rng = np.random.default_rng(seed)
    n_nodes = 4 * chunk + 64
    sizes = [1, 2, small_max, small_max + 1, chunk, chunk + 1, 3 * chunk + 5, max(1, small_max - 1)]
    sizes += list(rng.integers(1, small_max + 3, size=40))
    edges = [sorted(rng.choice(n_nodes - 8, size=s, replace=False).tolist()) for s in sizes]
    # a hub node in many hyperedges, a node with exactly small_max + 1, one
    # with small_max and one isolated (n_nodes - 1 never used)
    hub, a, b = n_nodes - 2, n_nodes - 3, n_nodes - 4
    deg_wanted = {hub: 2 * chunk + 7, a: small_max + 1, b: small_max}
    for node, k in deg_wanted.items():
        for _ in range(k):
            edges.append([node])
        # and membership in some bigger hyperedges too
        for e in rng.choice(len(sizes), size=3, replace=False):
            if node not in edges[e]:
                edges[e] = sorted(edges[e] + [node])
    ptr = np.concatenate([[0], np.cumsum([len(e) for e in edges])]).astype(np.int64)
    idx = np.array([v for e in edges for v in e], dtype=np.int32)
    w = rng.uniform(0.5, 2.0, size=len(edges)).astype(np.float32)
    from synth.hypergraph import Hypergraph
    return Hypergraph(n_nodes, len(edges), ptr, idx, w)


__all__ = ["CONFIGS", "coarsest_embedding", "make_hypergraph", "random_hypergraph", "rel_fro", "max_abs_rel",
           "assert_close", "assert_within", "assert_bf16", "bf16_reverse_bounds", "oracle_refine_bf16",
           "oracle_sweep_bf16", "BF16_U", "both_hierarchies", "tier_hypergraph"]
