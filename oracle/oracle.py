"""FP64 CPU oracle for HyperNetVec multi-level refinement (arXiv 2103.09660).

TEST INFRASTRUCTURE ONLY.  The oracle is the plain, slow reference the GPU
library is checked against.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` (which also reports the GPU results'
errors against it) may import it; the product package never
does.  It shares no code with the GPU library: the arithmetic lives in
``hnv_oracle.c`` (plain C, FP64) and the Python code below follows the paper's
three phases in order:

* Algorithm 1 (Section 3.1), one coarsening step per level, featureless or
  with bag-of-words node features (cosine assignment, merged feature rows);
* the projection rule at the end of Section 3.3 (a merged node's embedding is
  given to every fine node of its set);
* Algorithm 2 (Section 3.3), ``k`` smoothing sweeps per level, from the
  coarsest level to the finest;
* the reverse mode of the projection and of each sweep, and the linear
  cross-entropy head used downstream (Section 4, experimental settings);
* the hyperedge-prediction features (Section 4, hyperedge prediction): the
  per-dimension variance of a candidate set's member embeddings.

The function groups that have no external pin are listed under
``PARITY_UNPINNED`` below.  It is empty: every function, the early stop of
``refine`` included (``tests/test_oracle_early_stop.py``: a closed form of
the residual and the dense matrix chain), is pinned by a test in
``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess
from typing import List, Optional, Sequence

import numpy as np

PARITY_UNPINNED: tuple = ()

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hnv_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_f32p = ctypes.POINTER(ctypes.c_float)
_f64p = ctypes.POINTER(ctypes.c_double)


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (strict IEEE FP64, no contraction)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                               "-shared", "-fPIC", "-Wall", "-o", tmp, _SRC])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def _L():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB_PATH)
        lib.oracle_threads.restype = ctypes.c_int
        lib.oracle_set_threads.argtypes = [ctypes.c_int]
        lib.oracle_transpose.argtypes = [ctypes.c_int64, ctypes.c_int64, _i64p, _i32p, _i64p, _i32p]
        lib.oracle_coarsen.restype = ctypes.c_int
        lib.oracle_coarsen.argtypes = [ctypes.c_int64, ctypes.c_int64, _i64p, _i32p, _f32p, _i32p, _i32p,
                                       _i64p, _i64p, _i64p, _i64p, _i32p, _f32p]
        lib.oracle_coarsen_features.restype = ctypes.c_int
        lib.oracle_coarsen_features.argtypes = [ctypes.c_int64, ctypes.c_int64, _i64p, _i32p, _f32p, _i32p,
                                                ctypes.c_int, _i32p, _i32p, _i64p, _i64p, _i64p, _i64p, _i32p,
                                                _f32p, _i32p]
        lib.oracle_rowmap.argtypes = [ctypes.c_int64, ctypes.c_int64, _i64p, _i32p, _i32p, _i32p,
                                      ctypes.c_int64, _i64p]
        lib.oracle_project.argtypes = [ctypes.c_int64, _i64p, ctypes.c_int64, _f64p, _f64p]
        lib.oracle_sweep.argtypes = [ctypes.c_int64, ctypes.c_int64, _i64p, _i32p, _i64p, _i32p, _f32p,
                                     ctypes.c_int64, ctypes.c_double, ctypes.c_int, _f64p, _f64p]
        lib.oracle_sweep_vjp.argtypes = [ctypes.c_int64, ctypes.c_int64, _i64p, _i32p, _i64p, _i32p, _f32p,
                                         ctypes.c_int64, ctypes.c_double, _f64p, _f64p, _f64p, _f64p]
        lib.oracle_sweep_vjp_edge_first.argtypes = lib.oracle_sweep_vjp.argtypes
        lib.oracle_project_vjp.argtypes = [ctypes.c_int64, ctypes.c_int64, _i64p, ctypes.c_int64, _f64p, _f64p]
        _lib = lib
    return _lib


def threads() -> int:
    return int(_L().oracle_threads())


def set_threads(n: int) -> None:
    """Threads of the oracle's parallel loops from now on (timing only: the
    results do not depend on it)."""
    _L().oracle_set_threads(int(n))


def _p(a: Optional[np.ndarray], t):
    return None if a is None else a.ctypes.data_as(t)


@dataclasses.dataclass
class Level:
    """One hypergraph of the hierarchy, with both star-expansion adjacencies."""
    n_nodes: int
    n_edges: int
    eptr: np.ndarray                 # int64 [n_edges+1]  hyperedge -> members
    eidx: np.ndarray                 # int32 [nnz]
    w: Optional[np.ndarray]          # float32 [n_edges] or None (unit)
    nptr: np.ndarray = None          # int64 [n_nodes+1]  node -> hyperedges
    nidx: np.ndarray = None          # int32 [nnz]

    def __post_init__(self):
        self.eptr = np.ascontiguousarray(self.eptr, dtype=np.int64)
        self.eidx = np.ascontiguousarray(self.eidx, dtype=np.int32)
        if self.w is not None:
            self.w = np.ascontiguousarray(self.w, dtype=np.float32)
        if self.nptr is None:
            self.nptr, self.nidx = transpose(self.n_nodes, self.n_edges, self.eptr, self.eidx)

    @property
    def nnz(self) -> int:
        return int(self.eptr[-1])

    @property
    def rows(self) -> int:
        return self.n_nodes + self.n_edges


def transpose(n_nodes, n_edges, eptr, eidx):
    nptr = np.zeros(n_nodes + 1, dtype=np.int64)
    nidx = np.zeros(max(int(eptr[-1]), 1), dtype=np.int32)
    _L().oracle_transpose(n_nodes, n_edges, _p(eptr, _i64p), _p(eidx, _i32p), _p(nptr, _i64p), _p(nidx, _i32p))
    return nptr, nidx[: int(eptr[-1])]


@dataclasses.dataclass
class Coarsening:
    node_rep: np.ndarray   # int32 [n_nodes_fine]
    edge_rep: np.ndarray   # int32 [n_edges_fine], -1 = removed
    coarse: Level


def coarsen_level(lv: Level) -> Coarsening:
    """Algorithm 1's loop body once, featureless (Section 3.1)."""
    nnz = lv.nnz
    node_rep = np.zeros(max(lv.n_nodes, 1), dtype=np.int32)
    edge_rep = np.zeros(max(lv.n_edges, 1), dtype=np.int32)
    c_eptr = np.zeros(lv.n_edges + 1, dtype=np.int64)
    c_eidx = np.zeros(max(nnz, 1), dtype=np.int32)
    c_w = np.zeros(max(lv.n_edges, 1), dtype=np.float32)
    nv = ctypes.c_int64(); ne = ctypes.c_int64(); nz = ctypes.c_int64()
    rc = _L().oracle_coarsen(lv.n_nodes, lv.n_edges, _p(lv.eptr, _i64p), _p(lv.eidx, _i32p), _p(lv.w, _f32p),
                             _p(node_rep, _i32p), _p(edge_rep, _i32p), ctypes.byref(nv), ctypes.byref(ne),
                             ctypes.byref(nz), _p(c_eptr, _i64p), _p(c_eidx, _i32p), _p(c_w, _f32p))
    if rc != 0:
        raise MemoryError("oracle_coarsen")
    ne_, nz_ = ne.value, nz.value
    coarse = Level(nv.value, ne_, c_eptr[: ne_ + 1].copy(), c_eidx[:nz_].copy(),
                   None if lv.w is None else c_w[:ne_].copy())
    return Coarsening(node_rep[: lv.n_nodes].copy(), edge_rep[: lv.n_edges].copy(), coarse)


def coarsen_level_features(lv: Level, x: np.ndarray):
    """Algorithm 1's loop body once with node features (Section 3.1): x is
    the int32 [n_nodes x k] bag-of-words count matrix.  Returns
    (Coarsening, X' int32 [coarse n_nodes x k])."""
    x = np.ascontiguousarray(x, dtype=np.int32)
    assert x.ndim == 2 and x.shape[0] == lv.n_nodes
    k = x.shape[1]
    nnz = lv.nnz
    node_rep = np.zeros(max(lv.n_nodes, 1), dtype=np.int32)
    edge_rep = np.zeros(max(lv.n_edges, 1), dtype=np.int32)
    c_eptr = np.zeros(lv.n_edges + 1, dtype=np.int64)
    c_eidx = np.zeros(max(nnz, 1), dtype=np.int32)
    c_w = np.zeros(max(lv.n_edges, 1), dtype=np.float32)
    c_x = np.zeros((max(lv.n_nodes, 1), k), dtype=np.int32)
    nv = ctypes.c_int64(); ne = ctypes.c_int64(); nz = ctypes.c_int64()
    rc = _L().oracle_coarsen_features(lv.n_nodes, lv.n_edges, _p(lv.eptr, _i64p), _p(lv.eidx, _i32p),
                                      _p(lv.w, _f32p), _p(x, _i32p), k, _p(node_rep, _i32p), _p(edge_rep, _i32p),
                                      ctypes.byref(nv), ctypes.byref(ne), ctypes.byref(nz), _p(c_eptr, _i64p),
                                      _p(c_eidx, _i32p), _p(c_w, _f32p), _p(c_x, _i32p))
    if rc != 0:
        raise MemoryError("oracle_coarsen_features")
    ne_, nz_ = ne.value, nz.value
    coarse = Level(nv.value, ne_, c_eptr[: ne_ + 1].copy(), c_eidx[:nz_].copy(),
                   None if lv.w is None else c_w[:ne_].copy())
    return Coarsening(node_rep[: lv.n_nodes].copy(), edge_rep[: lv.n_edges].copy(), coarse), c_x[: nv.value].copy()


def build_hierarchy_features(n_nodes, n_edges, eptr, eidx, w, x, n_coarsen: int):
    """Levels 0 .. n_coarsen with feature-based coarsening; also returns the
    feature matrix of every level."""
    levels = [Level(n_nodes, n_edges, eptr, eidx, w)]
    feats = [np.ascontiguousarray(x, dtype=np.int32)]
    maps: List[Coarsening] = []
    for _ in range(n_coarsen):
        c, xc = coarsen_level_features(levels[-1], feats[-1])
        maps.append(c)
        levels.append(c.coarse)
        feats.append(xc)
    return levels, maps, feats


def build_hierarchy(n_nodes, n_edges, eptr, eidx, w, n_coarsen: int):
    """Levels 0 (finest) .. n_coarsen (coarsest) and the maps between them."""
    levels = [Level(n_nodes, n_edges, eptr, eidx, w)]
    maps: List[Coarsening] = []
    for _ in range(n_coarsen):
        c = coarsen_level(levels[-1])
        maps.append(c)
        levels.append(c.coarse)
    return levels, maps


def rowmap(fine: Level, cm: Coarsening) -> np.ndarray:
    out = np.zeros(fine.rows, dtype=np.int64)
    _L().oracle_rowmap(fine.n_nodes, fine.n_edges, _p(fine.eptr, _i64p), _p(fine.eidx, _i32p),
                       _p(cm.node_rep, _i32p), _p(cm.edge_rep, _i32p), cm.coarse.n_nodes, _p(out, _i64p))
    return out


def project(rmap: np.ndarray, zc: np.ndarray) -> np.ndarray:
    zc = np.ascontiguousarray(zc, dtype=np.float64)
    d = zc.shape[1]
    zf = np.empty((len(rmap), d), dtype=np.float64)
    _L().oracle_project(len(rmap), _p(rmap, _i64p), d, _p(zc, _f64p), _p(zf, _f64p))
    return zf


def sweep(lv: Level, z: np.ndarray, omega: float, order: int = 0, w: Optional[np.ndarray] = None) -> np.ndarray:
    """One iteration of Algorithm 2 over the star expansion of ``lv``.
    ``w`` overrides the level's hyperedge weights (e.g. learnt weights)."""
    z = np.ascontiguousarray(z, dtype=np.float64)
    assert z.shape[0] == lv.rows
    out = np.empty_like(z)
    ww = lv.w if w is None else np.ascontiguousarray(w, dtype=np.float32)
    _L().oracle_sweep(lv.n_nodes, lv.n_edges, _p(lv.eptr, _i64p), _p(lv.eidx, _i32p), _p(lv.nptr, _i64p),
                      _p(lv.nidx, _i32p), _p(ww, _f32p), z.shape[1], float(omega), int(order),
                      _p(z, _f64p), _p(out, _f64p))
    return out


def residual(z_new: np.ndarray, z_old: np.ndarray) -> float:
    """Frobenius norm of the change made by one sweep (the consecutive-
    iterate difference named as a stopping rule in Section 4)."""
    diff = np.asarray(z_new, dtype=np.float64) - np.asarray(z_old, dtype=np.float64)
    return float(np.sqrt(np.sum(diff * diff)))


def refine(levels: Sequence[Level], maps: Sequence[Coarsening], z_coarsest: np.ndarray,
           sweeps: Sequence[int], omega: float, order: int = 0, tol: float = 0.0,
           return_residuals: bool = False, return_counts: bool = False):
    """Refinement from the coarsest level to the finest (Section 3.3): sweeps
    at the coarsest level, then for each finer level project and sweep.
    ``sweeps[l]`` is the count for level l.

    ``tol > 0`` replaces the fixed count of a level by the stopping rule that
    Section 4 names as the alternative to a fixed iteration count: the
    level's sweeps end after the first sweep whose change
    ||Z^i - Z^(i-1)||_F (the whole level's matrix, absolute) is <= tol, or
    after ``sweeps[l]`` sweeps.  The rule is per level: the next finer level
    starts from the projection and runs its own sweeps.  The stopping
    sweep's residual is recorded.  Returns Z of level 0, plus the residuals
    (coarsest level first) and the sweeps run per level (index = level) when
    asked for."""
    L = len(levels) - 1
    z = np.ascontiguousarray(z_coarsest, dtype=np.float64)
    res = []
    counts = [0] * (L + 1)
    for lvl in range(L, -1, -1):
        if lvl < L:
            z = project(rowmap(levels[lvl], maps[lvl]), z)
        for _ in range(int(sweeps[lvl])):
            zn = sweep(levels[lvl], z, omega, order)
            r = residual(zn, z)
            res.append(r)
            counts[lvl] += 1
            z = zn
            if tol > 0 and r <= tol:
                break
    out = (z,)
    if return_residuals:
        out += (res,)
    if return_counts:
        out += (counts,)
    return out if len(out) > 1 else z


def sweep_vjp(lv: Level, y: np.ndarray, g: np.ndarray, omega: float, w: Optional[np.ndarray] = None,
              order: int = 0):
    """Reverse mode of one sweep at inputs ``y`` (order 0 Jacobi, order 1
    edge-first): returns (dL/dy, dL/dw)."""
    y = np.ascontiguousarray(y, dtype=np.float64)
    g = np.ascontiguousarray(g, dtype=np.float64)
    gy = np.empty_like(y)
    dw = np.zeros(max(lv.n_edges, 1), dtype=np.float64)
    ww = lv.w if w is None else np.ascontiguousarray(w, dtype=np.float32)
    fn = _L().oracle_sweep_vjp if order == 0 else _L().oracle_sweep_vjp_edge_first
    fn(lv.n_nodes, lv.n_edges, _p(lv.eptr, _i64p), _p(lv.eidx, _i32p), _p(lv.nptr, _i64p),
                          _p(lv.nidx, _i32p), _p(ww, _f32p), y.shape[1], float(omega), _p(y, _f64p),
                          _p(g, _f64p), _p(gy, _f64p), _p(dw, _f64p))
    return gy, dw[: lv.n_edges]


def project_vjp(rmap: np.ndarray, rows_coarse: int, gf: np.ndarray) -> np.ndarray:
    gf = np.ascontiguousarray(gf, dtype=np.float64)
    gc = np.empty((rows_coarse, gf.shape[1]), dtype=np.float64)
    _L().oracle_project_vjp(len(rmap), rows_coarse, _p(rmap, _i64p), gf.shape[1], _p(gf, _f64p), _p(gc, _f64p))
    return gc


def finest_refine_vjp(fine: Level, cm: Coarsening, z_coarse: np.ndarray, w: Optional[np.ndarray],
                      k: int, omega: float, g_out: np.ndarray, order: int = 0):
    """Forward and reverse of: project the coarse embedding onto the finest
    level, then ``k`` sweeps of the given order with hyperedge weights ``w``.
    Returns (Z_k, dL/dZ_coarse, dL/dw) for the cotangent ``g_out`` = dL/dZ_k."""
    rm = rowmap(fine, cm)
    states = [project(rm, z_coarse)]
    for _ in range(k):
        states.append(sweep(fine, states[-1], omega, order, w))
    g = np.ascontiguousarray(g_out, dtype=np.float64)
    dw = np.zeros(fine.n_edges, dtype=np.float64)
    for i in range(k, 0, -1):
        g, dwi = sweep_vjp(fine, states[i - 1], g, omega, w, order)
        dw += dwi
    gc = project_vjp(rm, cm.coarse.rows, g)
    return states[-1], gc, dw


def ce_head(z_nodes: np.ndarray, labels: np.ndarray, W: np.ndarray, b: np.ndarray):
    """Mean cross-entropy of a linear head, FP64: returns (loss, dL/dz_nodes).
    logits = z W^T + b; loss = mean_i (logsumexp(logits_i) - logits_i[y_i])."""
    z = np.asarray(z_nodes, dtype=np.float64)
    W64 = np.asarray(W, dtype=np.float64)
    logits = z @ W64.T + np.asarray(b, dtype=np.float64)
    m = logits.max(axis=1, keepdims=True)
    ex = np.exp(logits - m)
    se = ex.sum(axis=1, keepdims=True)
    lse = (m + np.log(se))[:, 0]
    n = len(labels)
    loss = float(np.mean(lse - logits[np.arange(n), labels]))
    p = ex / se
    p[np.arange(n), labels] -= 1.0
    dz = (p / n) @ W64
    return loss, dz


def score_candidates(z_nodes: np.ndarray, cand_ptr: np.ndarray, cand_idx: np.ndarray, op: str = "variance"):
    """Hyperedge-prediction features (Section 4, hyperedge prediction): for
    each candidate node set, a per-dimension statistic of its members' rows
    in FP64 -- the population variance (the paper's operator), or the mean,
    min or max it names as alternatives.  The variance is computed in two
    passes, mean first, then the mean squared deviation.  Empty sets and
    member ids outside the matrix give NaN rows."""
    z = np.asarray(z_nodes, dtype=np.float64)
    n_cand = len(cand_ptr) - 1
    out = np.full((n_cand, z.shape[1]), np.nan)
    for c in range(n_cand):
        members = np.asarray(cand_idx[cand_ptr[c]:cand_ptr[c + 1]], dtype=np.int64)
        if len(members) == 0 or members.min() < 0 or members.max() >= z.shape[0]:
            continue
        rows = z[members]
        if op == "variance":
            mean = rows.sum(axis=0) / len(members)
            out[c] = ((rows - mean) ** 2).sum(axis=0) / len(members)
        elif op == "mean":
            out[c] = rows.sum(axis=0) / len(members)
        elif op == "min":
            out[c] = rows.min(axis=0)
        elif op == "max":
            out[c] = rows.max(axis=0)
        else:
            raise ValueError(op)
    return out
