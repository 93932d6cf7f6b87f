"""Property-based checks (hypothesis) of the library's host coarsening on
tiny random hypergraphs: bit-exact against the oracle and against the
independent brute-force re-derivation, and every malformed level rejected
with its status."""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

from tests.test_oracle_coarsen import brute_force_coarsen


@pytest.fixture(scope="module")
def H():
    import paper_2103_09660_amd as H
    H.abi_version()
    return H


@st.composite
def hypergraphs(draw):
    n = draw(st.integers(1, 12))
    m = draw(st.integers(0, 10))
    edges = [sorted(draw(st.sets(st.integers(0, n - 1), min_size=1, max_size=min(4, n)))) for _ in range(m)]
    weighted = draw(st.booleans())
    w = [float(draw(st.sampled_from([1.0, 2.0, 3.0]))) for _ in range(m)] if weighted else None
    return n, edges, w


def _arrays(edges):
    ptr = np.concatenate([[0], np.cumsum([len(e) for e in edges])]).astype(np.int64)
    idx = np.array([v for e in edges for v in e], dtype=np.int32)
    return ptr, idx


@settings(max_examples=200, deadline=None, suppress_health_check=[HealthCheck.function_scoped_fixture])
@given(g=hypergraphs())
def test_host_coarsening_matches_oracle_and_brute_force(oracle_mod, H, g):
    n, edges, w = g
    ptr, idx = _arrays(edges)
    wa = None if w is None else np.array(w, dtype=np.float32)
    m, c = H.coarsen_level(H.HostLevel(n, len(edges), ptr, idx, wa))
    ref = oracle_mod.coarsen_level(oracle_mod.Level(n, len(edges), ptr, idx, wa))
    assert np.array_equal(m.node_rep, ref.node_rep) and np.array_equal(m.edge_rep, ref.edge_rep)
    assert np.array_equal(c.edge_ptr, ref.coarse.eptr) and np.array_equal(c.edge_idx, ref.coarse.eidx)
    rep, erep, n_c, coarse, cw = brute_force_coarsen(n, [set(e) for e in edges], w or [1.0] * len(edges))
    assert m.node_rep.tolist() == rep and m.edge_rep.tolist() == erep and c.n_nodes == n_c
    got = [c.edge_idx[c.edge_ptr[i]:c.edge_ptr[i + 1]].tolist() for i in range(c.n_edges)]
    assert got == coarse


@settings(max_examples=150, deadline=None, suppress_health_check=[HealthCheck.function_scoped_fixture])
@given(g=hypergraphs(), data=st.data())
def test_malformed_levels_get_their_status(H, g, data):
    from paper_2103_09660_amd import _lib as L
    n, edges, w = g
    if not edges:
        return
    ptr, idx = _arrays(edges)
    kind = data.draw(st.sampled_from(["range", "order", "weight", "empty"]))
    wa = None if w is None else np.array(w, dtype=np.float32)
    if kind == "range":
        idx[data.draw(st.integers(0, len(idx) - 1))] = data.draw(st.sampled_from([-1, n, n + 5]))
        want = L.HNV_ERANGE
    elif kind == "order":
        big = [e for e in range(len(edges)) if len(edges[e]) >= 2]
        if not big:
            return
        e = data.draw(st.sampled_from(big))
        a = int(ptr[e])
        idx[a], idx[a + 1] = idx[a + 1], idx[a]
        want = L.HNV_EUNSORTED
    elif kind == "weight":
        wa = np.ones(len(edges), dtype=np.float32)
        wa[data.draw(st.integers(0, len(edges) - 1))] = data.draw(st.sampled_from([0.0, -1.0, float("nan"),
                                                                                    float("inf")]))
        want = L.HNV_EINVAL
    else:
        e = data.draw(st.integers(0, len(edges) - 1))
        edges = edges[:e] + [[]] + edges[e:]
        ptr, idx = _arrays(edges)
        wa = None
        want = L.HNV_EINVAL
    with pytest.raises(H.HnvError) as ei:
        H.validate_level(H.HostLevel(n, len(edges), ptr, idx, wa))
    assert ei.value.status == want
