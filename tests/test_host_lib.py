"""Host-side tests of the library (no GPU needed): the shared object loads and
exports every call declared in include/hnv.h, input validation returns the
documented status codes, and the library's own coarsening (Section 3.1,
Algorithm 1) is bit-exact with the oracle's."""
import ctypes
import os
import re

import numpy as np
import pytest

from tests.cases import CONFIGS, make_hypergraph, random_hypergraph

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def H():
    import paper_2103_09660_amd as H
    return H


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "hnv.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hnv_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_call(H):
    from paper_2103_09660_amd import _lib
    names = _declared_functions()
    assert len(names) >= 17
    lib = ctypes.CDLL(_lib.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(_lib.exported_names()) == names
    assert H.abi_version() == 2


def _lvl(H, n_nodes, edges, w=None):
    ptr = np.concatenate([[0], np.cumsum([len(e) for e in edges])]).astype(np.int64)
    idx = np.array([v for e in edges for v in e], dtype=np.int32)
    return H.HostLevel(n_nodes, len(edges), ptr, idx, None if w is None else np.asarray(w, np.float32))


def test_validation_status_codes(H):
    from paper_2103_09660_amd._lib import HNV_EINVAL, HNV_ERANGE, HNV_EUNSORTED, HnvError
    H.validate_level(_lvl(H, 4, [[0, 1], [2, 3]]))
    cases = [
        (_lvl(H, 4, [[0, 4]]), HNV_ERANGE),
        (_lvl(H, 4, [[1, 0]]), HNV_EUNSORTED),
        (_lvl(H, 4, [[1, 1]]), HNV_EUNSORTED),
        (_lvl(H, 4, [[0], []]), HNV_EINVAL),
        (_lvl(H, 4, [[0, 1]], w=[0.0]), HNV_EINVAL),
        (_lvl(H, 4, [[0, 1]], w=[np.inf]), HNV_EINVAL),
        (_lvl(H, 4, [[0, 1]], w=[-1.0]), HNV_EINVAL),
    ]
    for lv, code in cases:
        with pytest.raises(HnvError) as ei:
            H.validate_level(lv)
        assert ei.value.status == code, str(ei.value)
        assert H.last_error() != ""
        with pytest.raises(HnvError):
            H.coarsen_level(lv)


def _csc(n_nodes, ptr, idx):
    """The transpose written out from its definition: node v's hyperedges in
    ascending id."""
    lists = [[] for _ in range(n_nodes)]
    for e in range(len(ptr) - 1):
        for j in range(ptr[e], ptr[e + 1]):
            lists[idx[j]].append(e)
    nptr = np.concatenate([[0], np.cumsum([len(x) for x in lists])]).astype(np.int64)
    nidx = np.array([e for x in lists for e in x], dtype=np.int32)
    return nptr, nidx


def test_caller_csc_is_checked_as_the_exact_transpose(H):
    """A level may carry its CSC (node -> hyperedges); it must be the exact
    transpose of the CSR, and a plan sized from it is the one sized from the
    CSR alone."""
    import dataclasses
    from paper_2103_09660_amd._lib import HNV_EINVAL, HnvError
    hg = random_hypergraph(4, 300, 200, 1, 9, weighted=True)
    nptr, nidx = _csc(hg.n_nodes, hg.edge_ptr, hg.edge_idx)
    base = H.HostLevel(hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, hg.edge_w)
    good = dataclasses.replace(base, node_ptr=nptr, node_idx=nidx)
    H.validate_level(good)
    bad = []
    swapped = nidx.copy()                       # a list out of order
    v = int(np.argmax(np.diff(nptr) >= 2))
    swapped[nptr[v]], swapped[nptr[v] + 1] = swapped[nptr[v] + 1], swapped[nptr[v]]
    bad.append(("unsorted list", nptr, swapped))
    wrong = nidx.copy()                         # a hyperedge that does not hold the node
    wrong[nptr[v]] = (wrong[nptr[v]] + 1) % hg.n_edges
    bad.append(("foreign hyperedge", nptr, wrong))
    moved = nptr.copy()                         # an entry moved to the next node
    moved[v + 1] -= 1
    bad.append(("shifted offsets", moved, nidx))
    short = nptr.copy()
    short[-1] -= 1
    bad.append(("does not end at nnz", short, nidx))
    for what, p, i in bad:
        with pytest.raises(HnvError) as ei:
            H.validate_level(dataclasses.replace(base, node_ptr=p, node_idx=i))
        assert ei.value.status == HNV_EINVAL, what
    with pytest.raises(HnvError) as ei:
        H.validate_level(dataclasses.replace(base, node_ptr=nptr))
    assert ei.value.status == HNV_EINVAL
    # the plan's size does not depend on where the CSC comes from
    hier = H.Hierarchy.build(hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, hg.edge_w, 1)
    with_csc = H.Hierarchy([dataclasses.replace(hier.levels[0], node_ptr=nptr, node_idx=nidx)] + hier.levels[1:],
                           hier.maps)
    for d, dt in ((64, "bf16"), (32, "f32")):
        assert H.plan_workspace_bytes(with_csc, d, dt) == H.plan_workspace_bytes(hier, d, dt)
    # sizing reads the CSC's offsets, so they are checked there too
    dec = nptr.copy()
    dec[v + 1] = dec[v] - 1
    bad_hier = H.Hierarchy([dataclasses.replace(hier.levels[0], node_ptr=dec, node_idx=nidx)] + hier.levels[1:],
                           hier.maps)
    with pytest.raises(HnvError) as ei:
        H.plan_workspace_bytes(bad_hier, 64, "bf16")
    assert ei.value.status == HNV_EINVAL


def test_workspace_sizing_errors(H):
    from paper_2103_09660_amd._lib import HNV_EUNSUPPORTED, HnvError
    hg = random_hypergraph(0, 40, 20, 1, 4)
    hier = H.Hierarchy.build(hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, hg.edge_w, 1)
    assert H.plan_workspace_bytes(hier, 64, "bf16") > 0
    for d in (0, 12, 520):
        with pytest.raises(HnvError) as ei:
            H.plan_workspace_bytes(hier, d, "f32")
        assert ei.value.status == HNV_EUNSUPPORTED
    with pytest.raises(HnvError):
        H.plan_workspace_bytes(hier, 64, "f32", options={"panel_cols": 24})
    # a coarser level with more rows than the finest would not fit the
    # refinement's buffers (a valid map onto a level with unused nodes)
    fine = _lvl(H, 4, [[0, 1], [2, 3]])
    big = _lvl(H, 6, [[0, 1]])
    grown = H.Hierarchy([fine, big], [H.HostMap(np.array([0, 0, 1, 1], np.int32), np.array([0, -1], np.int32))])
    with pytest.raises(HnvError) as ei:
        H.plan_workspace_bytes(grown, 16, "f32")
    assert ei.value.status == HNV_EUNSUPPORTED and "more rows than level 0" in str(ei.value)
    # more panels / smaller tiers never shrink below the embedding buffer
    a = H.plan_workspace_bytes(hier, 64, "f32", options={"panel_cols": 32, "small_max": 1, "chunk": 64})
    assert a >= hier.levels[0].rows * 64 * 4


@pytest.mark.parametrize("seed", range(30))
def test_coarsening_bit_exact_random(oracle_mod, H, seed):
    O = oracle_mod
    hg = random_hypergraph(seed, 5 + 3 * seed, 4 + 2 * seed, 1, 7, weighted=(seed % 3 != 0),
                           integer_weights=(seed % 3 == 1))
    lv = O.Level(hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, hg.edge_w)
    for _ in range(3):
        c = O.coarsen_level(lv)
        m, co = H.coarsen_level(H.HostLevel(lv.n_nodes, lv.n_edges, lv.eptr, lv.eidx, lv.w))
        assert np.array_equal(m.node_rep, c.node_rep) and np.array_equal(m.edge_rep, c.edge_rep)
        assert (co.n_nodes, co.n_edges) == (c.coarse.n_nodes, c.coarse.n_edges)
        assert np.array_equal(co.edge_ptr, c.coarse.eptr) and np.array_equal(co.edge_idx, c.coarse.eidx)
        if lv.w is not None:
            assert np.array_equal(co.edge_w, c.coarse.w)
        lv = c.coarse


@pytest.mark.parametrize("name", ["tiny-2k", "hub-200k"])
def test_coarsening_bit_exact_configs(oracle_mod, H, name):
    from tests.cases import both_hierarchies
    cfg = CONFIGS[name]
    both_hierarchies(oracle_mod, H, make_hypergraph(cfg), cfg.levels)


def test_missing_library_fails_loudly(tmp_path, monkeypatch):
    """The binding has no fallback: without the shared object it raises."""
    from paper_2103_09660_amd import _lib
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "absent.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(ImportError):
        _lib.lib()


@pytest.mark.parametrize("seed,small_max,chunk", [(11, 4, 64), (11, 8, 64), (11, 32, 128), (11, 1, 64),
                                                  (5, 8, 64), (1, 4, 64), (3, 8, 128)])
def test_tier_inputs_are_valid_and_coarsen_identically(oracle_mod, H, seed, small_max, chunk):
    """The tier-boundary inputs used by the GPU tests are valid hypergraphs and
    both hierarchies agree on them (checked here, without a GPU)."""
    from tests.cases import both_hierarchies, tier_hypergraph
    hg = tier_hypergraph(seed, small_max, chunk)
    H.validate_level(H.HostLevel(hg.n_nodes, hg.n_edges, hg.edge_ptr, hg.edge_idx, hg.edge_w))
    both_hierarchies(oracle_mod, H, hg, 2)


def test_size_limits_rejected_before_any_read(H):
    """Levels of 2^31 incidences or star-expansion rows are refused with
    HNV_EUNSUPPORTED from their sizes alone: the arrays passed are far
    shorter than the sizes claim and are never read past their ends."""
    import ctypes
    from paper_2103_09660_amd import _lib as L
    lib = L.lib()
    big = 1 << 31
    ptr = (ctypes.c_int64 * 2)(0, big)
    idx = (ctypes.c_int32 * 1)(0)
    size = ctypes.c_size_t()
    for n_nodes, n_edges, nnz in ((4, 1, big), (big - 1, 1, 2), (big, 1, 2)):
        lv = L.HnvLevel(n_nodes, n_edges, nnz, ctypes.cast(ptr, L.i64p), ctypes.cast(idx, L.i32p), None)
        assert lib.hnv_validate_level(ctypes.byref(lv)) == L.HNV_EUNSUPPORTED, (n_nodes, n_edges, nnz)
        assert "2^31" in H.last_error()
        assert lib.hnv_plan_workspace_bytes(ctypes.byref(lv), None, 1, 64, 0, None,
                                            ctypes.byref(size)) == L.HNV_EUNSUPPORTED
        # the GPU coarsening's sizing refuses them before it queries any device
        assert lib.hnv_coarsen_workspace_bytes(n_nodes, n_edges, nnz, ctypes.byref(size)) == L.HNV_EUNSUPPORTED
    # a small valid level passes the same checks
    lv = L.HnvLevel(4, 1, 2, ctypes.cast((ctypes.c_int64 * 2)(0, 2), L.i64p),
                    ctypes.cast((ctypes.c_int32 * 2)(0, 1), L.i32p), None)
    assert lib.hnv_validate_level(ctypes.byref(lv)) == L.HNV_OK

