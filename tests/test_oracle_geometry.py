"""Pins for the oracle's cell traversal against brute-force slab geometry.

The march advances one cell at a time (Alg. functors raymarch, Amanatides-Woo
traversal); rays leave a non-periodic box, and in a periodic box wrap and
stop once they have travelled sqrt(3) L_box (Sec. "Periodic BCs").
"""
import math

import numpy as np
import pytest

from bruteforce import box_exit, cells_along


def _unit(v):
    v = np.asarray(v, float)
    return v / np.linalg.norm(v)


def _rays(seed, k, n):
    g = np.random.default_rng(seed)
    o = g.random((k, 3)) * n
    d = g.standard_normal((k, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    return o, d


def _log_one(orc, n, periodic, o, d):
    p = orc.make_params(n, 1.0e20, periodic=periodic, n_min_ray=0.0, corr=orc.CORR_NONE)
    nH = np.full((n, n, n), 1e-6)
    x = np.zeros((n, n, n))
    _, b, log = orc.trace_rays(p, nH, x, o[None], d[None], 0, 1.0, max_log=100000)
    assert log["count"] == b["segments"]
    return log, b


@pytest.mark.parametrize("seed", range(6))
def test_dda_matches_slab_method_open_box(orc, seed):
    n = 8
    o, d = _rays(100 + seed, 20, n)
    for r in range(o.shape[0]):
        log, _ = _log_one(orc, n, False, o[r], d[r])
        s_exit = box_exit(o[r], d[r], n)
        ref = cells_along(o[r], d[r], 0.0, s_exit)
        keep = log["ds"] > 1e-9
        got_cells = [tuple(c) for c in log["ijk"][keep]]
        assert got_cells == [c for c, _, _ in ref]
        np.testing.assert_allclose(log["ds"][keep], [t1 - t0 for _, t0, t1 in ref],
                                   rtol=0, atol=1e-12)
        assert abs(log["ds"].sum() - s_exit) < 1e-12 * n


@pytest.mark.parametrize("seed", range(3))
def test_dda_matches_slab_method_periodic(orc, seed):
    """Unwrapped cells up to sqrt(3) n; wrapped flat index = cell mod n."""
    n = 6
    o, d = _rays(200 + seed, 10, n)
    s_max = math.sqrt(3.0) * n
    for r in range(o.shape[0]):
        log, b = _log_one(orc, n, True, o[r], d[r])
        ref = cells_along(o[r], d[r], 0.0, s_max)
        keep = log["ds"] > 1e-9
        ijk = log["ijk"][keep]
        assert [tuple(c) for c in ijk] == [c for c, _, _ in ref]
        np.testing.assert_allclose(log["ds"][keep], [t1 - t0 for _, t0, t1 in ref], atol=1e-12)
        w = np.mod(ijk, n)
        np.testing.assert_array_equal(log["cell"][keep], w[:, 0] + n * (w[:, 1] + n * w[:, 2]))
        # the march ends at the first cell boundary at or beyond sqrt(3) n
        total = log["ds"].sum()
        assert total >= s_max - 1e-12 and total - s_max <= math.sqrt(3.0) + 1e-12
        assert b["escaped"] > 0 and b["truncated"] == 0


def test_structured_ties(orc):
    """Rays through cell corners from a cell centre: the traversal takes the
    exact diagonal cells, with a zero-length segment at each tie."""
    n = 8
    o = np.array([0.5, 0.5, 0.5])
    for d in ([1, 1, 0], [1, 1, 1], [1, 0, 0], [-1, 1, 0], [0, -1, -1]):
        d = _unit(d)
        oo = o.copy()
        oo[d < 0] = n - 0.5
        log, _ = _log_one(orc, n, False, oo, d)
        ref = cells_along(oo, d, 0.0, box_exit(oo, d, n))
        keep = log["ds"] > 1e-9
        assert [tuple(c) for c in log["ijk"][keep]] == [c for c, _, _ in ref]
        nz = int((~keep).sum())
        nonzero_axes = int((d != 0).sum())
        assert nz == (len(ref) - 1) * (nonzero_axes - 1) or len(ref) <= 1


def test_start_on_boundary_with_negative_direction(orc):
    """A start point exactly on a cell face with a negative component starts
    in the cell below (the ray is leaving the upper cell)."""
    n = 4
    o = np.array([2.0, 1.5, 1.5])
    d = np.array([-1.0, 0.0, 0.0])
    log, _ = _log_one(orc, n, False, o, d)
    assert tuple(log["ijk"][0]) == (1, 1, 1)
    np.testing.assert_allclose(log["ds"], [1.0, 1.0])
    log, _ = _log_one(orc, n, False, o, -d)
    assert tuple(log["ijk"][0]) == (2, 1, 1)
