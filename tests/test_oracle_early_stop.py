"""Pins for the oracle's early stop (the epsilon rule that Section 4 names as
the alternative to a fixed count of refinement iterations): per level, the
sweeps end after the first sweep whose change ||Z^i - Z^(i-1)||_F is at most
tol, or after the level's sweep count.

The stopping sweep is derived here without the oracle's loop: from a closed
form of the residual for one hyperedge, and from the dense matrix chain of
the paper's Section 3.3 statement (projection, then relaxed Jacobi steps on
L z = 0) over a whole hierarchy.  Both compare the sweeps run per level, the
residual of every sweep and the final embedding, so a misreading of the rule
(stopping the whole refinement instead of the level, testing before the
residual is recorded, a relative instead of an absolute test) fails here."""
import numpy as np
import pytest

from synth import random_hypergraph
from tests.dense_ref import jacobi_matrix, projection_matrix, star_adjacency


def _closed_form_residuals(z0, n, omega, K):
    """One hyperedge of n members (rows 0..n-1 the members, row n the
    hyperedge), Jacobi.  With m0 the member mean and e0 the hyperedge row,
    e_i - e_(i-1) = -omega (1-2 omega)^(i-1) (e0 - m0) and
    z_u,i - z_u,(i-1) = omega (1-2 omega)^(i-1) (e0 - m0) - omega (1-omega)^(i-1) (z_u,0 - m0).
    The members' deviations from m0 sum to zero, so the cross term vanishes:
    rho_i^2 = omega^2 [(n+1) (1-2 omega)^(2(i-1)) |e0-m0|^2 + (1-omega)^(2(i-1)) sum_u |z_u,0-m0|^2]."""
    m0 = z0[:n].mean(axis=0)
    a = float(np.sum((z0[n] - m0) ** 2))
    b = float(np.sum((z0[:n] - m0) ** 2))
    out = []
    for i in range(1, K + 1):
        p = (1 - 2 * omega) ** (2 * (i - 1)) if i > 1 else 1.0
        q = (1 - omega) ** (2 * (i - 1))
        out.append(omega * np.sqrt((n + 1) * p * a + q * b))
    return np.array(out)


def _closed_form_state(z0, n, omega, i):
    m0 = z0[:n].mean(axis=0)
    e0 = z0[n]
    z = np.empty_like(z0)
    z[n] = (m0 + e0) / 2 + (1 - 2 * omega) ** i * (e0 - m0) / 2
    z[:n] = (m0 + e0) / 2 - (1 - 2 * omega) ** i * (e0 - m0) / 2 + (1 - omega) ** i * (z0[:n] - m0)
    return z


@pytest.mark.parametrize("omega", [0.5, 0.25, 0.8])
def test_early_stop_single_hyperedge_closed_form(oracle_mod, omega):
    O = oracle_mod
    n, K = 9, 30
    lv = O.Level(n, 1, np.array([0, n]), np.arange(n, dtype=np.int32), None)
    z0 = np.random.default_rng(5).standard_normal((n + 1, 3))
    rho = _closed_form_residuals(z0, n, omega, K)
    assert np.all(np.diff(rho) < 0)       # strictly decreasing for 0 < omega < 1
    # without a tol every sweep runs and every residual is the closed form
    z, res, counts = O.refine([lv], [], z0, [K], omega, return_residuals=True, return_counts=True)
    assert counts == [K]
    # differences of rounded iterates: absolute floor at the rounding of Z
    atol = 1e-14 * float(np.abs(z0).max())
    np.testing.assert_allclose(res, rho, rtol=1e-11, atol=atol)
    for k in (1, 3, 7):
        # tol between rho_k and rho_(k+1): the level stops after sweep k+1,
        # whose residual is the first at or below tol and is recorded
        tol = float(np.sqrt(rho[k - 1] * rho[k]))
        z, res, counts = O.refine([lv], [], z0, [K], omega, tol=tol, return_residuals=True,
                                  return_counts=True)
        assert counts == [k + 1]
        np.testing.assert_allclose(res, rho[: k + 1], rtol=1e-11, atol=atol)
        np.testing.assert_allclose(z, _closed_form_state(z0, n, omega, k + 1), rtol=0, atol=1e-13)
    # a tol above the first change stops after one sweep; one below every
    # change runs the count; the test is on the absolute change, so scaling
    # Z and tol together changes nothing
    assert O.refine([lv], [], z0, [K], omega, tol=2 * rho[0], return_counts=True)[1] == [1]
    assert O.refine([lv], [], z0, [K], omega, tol=0.5 * rho[-1], return_counts=True)[1] == [K]
    tol = float(np.sqrt(rho[4] * rho[5]))
    assert O.refine([lv], [], 1e3 * z0, [K], omega, tol=1e3 * tol, return_counts=True)[1] == [6]
    assert O.refine([lv], [], 1e3 * z0, [K], omega, tol=tol, return_counts=True)[1] != [6]


def _dense_refine_early_stop(O, levels, maps, zc, K, omega, tol):
    """The refinement as dense matrices: per level (coarsest first) the
    projection matrix, then up to K[l] applications of the relaxed Jacobi
    matrix I - omega D^-1 L, stopping the level after the first change of
    Frobenius norm <= tol."""
    L = len(levels) - 1
    z = np.asarray(zc, dtype=np.float64)
    res, counts = [], [0] * (L + 1)
    for lvl in range(L, -1, -1):
        lv = levels[lvl]
        if lvl < L:
            z = projection_matrix(O.rowmap(lv, maps[lvl]), levels[lvl + 1].rows) @ z
        M = jacobi_matrix(star_adjacency(lv.n_nodes, lv.n_edges, lv.eptr, lv.eidx, lv.w), omega)
        for _ in range(K[lvl]):
            zn = M @ z
            r = float(np.linalg.norm(zn - z))
            res.append(r)
            counts[lvl] += 1
            z = zn
            if r <= tol:
                break
    return z, res, counts


@pytest.mark.parametrize("seed,omega", [(3, 0.5), (8, 0.35), (12, 0.7)])
def test_early_stop_per_level_dense_chain(oracle_mod, seed, omega):
    O = oracle_mod
    hg = random_hypergraph(seed, 60, 40, 1, 6, weighted=True)
    levels, maps = O.build_hierarchy(hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, hg.edge_w, 3)
    L = len(levels) - 1
    K = [25] * (L + 1)
    zc = np.random.default_rng(seed).standard_normal((levels[L].rows, 4))
    _, free_res, _ = _dense_refine_early_stop(O, levels, maps, zc, K, omega, 0.0)
    checked = 0
    for q in (0.3, 0.5, 0.7, 0.85):
        tol = float(np.quantile(free_res, q))
        z_ref, res_ref, cnt_ref = _dense_refine_early_stop(O, levels, maps, zc, K, omega, tol)
        # decisions this close to tol could flip with rounding: move tol off them
        while min(abs(r - tol) for r in res_ref) <= 1e-8 * tol:
            tol *= 1.01
            z_ref, res_ref, cnt_ref = _dense_refine_early_stop(O, levels, maps, zc, K, omega, tol)
        z, res, cnt = O.refine(levels, maps, zc, K, omega, tol=tol, return_residuals=True, return_counts=True)
        assert cnt == cnt_ref, (tol, cnt, cnt_ref)
        np.testing.assert_allclose(res, res_ref, rtol=1e-10)
        assert np.linalg.norm(z - z_ref) <= 1e-12 * np.linalg.norm(z_ref)
        # an informative case: a level coarser than the finest stops early,
        # and the finer levels still sweep after it (every level runs at
        # least one sweep, so stopping the whole refinement would differ)
        if any(cnt_ref[l] < K[l] for l in range(1, L + 1)):
            checked += 1
    assert checked >= 1


def test_early_stop_off_runs_fixed_counts(oracle_mod):
    O = oracle_mod
    hg = random_hypergraph(2, 40, 25, 1, 5, weighted=False)
    levels, maps = O.build_hierarchy(hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, None, 2)
    zc = np.random.default_rng(2).standard_normal((levels[2].rows, 2))
    K = [3, 0, 5]
    for tol in (0.0, -1.0):
        z, res, cnt = O.refine(levels, maps, zc, K, 0.5, tol=tol, return_residuals=True, return_counts=True)
        assert cnt == K and len(res) == sum(K)
        z_ref, res_ref, cnt_ref = _dense_refine_early_stop(O, levels, maps, zc, K, 0.5, -np.inf)
        assert cnt_ref == K
        np.testing.assert_allclose(res, res_ref, rtol=1e-10)
        assert np.linalg.norm(z - z_ref) <= 1e-12 * np.linalg.norm(z_ref)
