"""Pins for the oracle's hyperedge-prediction features (Section 4): the
population variance against a library routine and closed forms, and the
mean / min / max alternatives."""
import statistics

import numpy as np
import pytest


def _csr(sets):
    ptr = np.concatenate([[0], np.cumsum([len(s) for s in sets])]).astype(np.int64)
    idx = np.array([v for s in sets for v in s], dtype=np.int64)
    return ptr, idx


def test_variance_closed_forms_and_library(oracle_mod):
    O = oracle_mod
    rng = np.random.default_rng(0)
    z = rng.standard_normal((50, 6))
    delta = rng.standard_normal(6)
    z[10] = z[11] + delta
    sets = [[11, 10], [3], [4, 7, 9, 20, 33], list(range(50))]
    ptr, idx = _csr(sets)
    var = O.score_candidates(z, ptr, idx, "variance")
    np.testing.assert_allclose(var[0], delta ** 2 / 4, rtol=1e-14)        # two points
    np.testing.assert_array_equal(var[1], np.zeros(6))                    # one point
    for c, s in enumerate(sets):
        for j in range(6):
            assert abs(var[c, j] - statistics.pvariance(z[s, j].tolist())) <= 1e-13
    # translation invariance of the variance, equivariance of the others
    shift = rng.standard_normal(6)
    np.testing.assert_allclose(O.score_candidates(z + shift, ptr, idx, "variance"), var, atol=1e-13)
    mean = O.score_candidates(z, ptr, idx, "mean")
    np.testing.assert_allclose(O.score_candidates(z + shift, ptr, idx, "mean"), mean + shift, atol=1e-13)
    for c, s in enumerate(sets):
        np.testing.assert_array_equal(O.score_candidates(z, ptr, idx, "min")[c], np.min(z[s], axis=0))
        np.testing.assert_array_equal(O.score_candidates(z, ptr, idx, "max")[c], np.max(z[s], axis=0))
        np.testing.assert_allclose(mean[c], [statistics.fmean(z[s, j].tolist()) for j in range(6)], atol=1e-14)


@pytest.mark.parametrize("op", ["variance", "mean", "min", "max"])
def test_invalid_sets_are_nan(oracle_mod, op):
    O = oracle_mod
    z = np.ones((5, 2))
    ptr, idx = _csr([[], [1, 7], [0, 2]])
    out = O.score_candidates(z, ptr, idx, op)
    assert np.isnan(out[0]).all() and np.isnan(out[1]).all() and not np.isnan(out[2]).any()
