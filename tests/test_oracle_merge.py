"""Pins for the oracle's source merging (Sec. "Source Merging Algorithm",
Alg. source_merge).

* Same-cell sources merge by summing rates; the catalogue is sorted.
* max_radius on a single spherical bubble of radius R_b around the source:
  a shell sample at distance r lands in a cell whose centre is within
  r +- sqrt(3)/2, so every shell with r <= R_b - sqrt(3)/2 passes and every
  shell with r > R_b + sqrt(3)/2 fails; the radius therefore lies in
  (R_b - sqrt(3)/2 - dr, R_b + sqrt(3)/2].  A neutral source cell gives 0,
  an ionized box gives R_max.
* The groups are the connected components of the overlap graph, computed
  here by breadth-first search over all pairs; each merged source carries
  the group's total rate and largest radius and sits on one of the group's
  cells; the output is sorted lexicographically.
"""
import math
from collections import deque

import numpy as np
import pytest

import workloads as W


def test_dedupe_and_sort(orc):
    n = 16
    pos = np.array([[3.2, 1.1, 9.9], [0.5, 5.5, 2.5], [3.9, 1.8, 9.0], [0.1, 5.0, 2.0],
                    [15.9, 0.0, 0.0]])
    ndot = np.array([1.0, 2.0, 4.0, 8.0, 16.0])
    cells, flux = orc.dedupe_sort(n, pos, ndot)
    np.testing.assert_array_equal(cells, [[0, 5, 2], [3, 1, 9], [15, 0, 0]])
    np.testing.assert_array_equal(flux, [10.0, 5.0, 16.0])


@pytest.mark.parametrize("rb", [3.0, 4.5, 6.0, 7.3, 9.0])
def test_max_radius_single_bubble(orc, rb):
    n = 40
    mp = orc.make_merge_params(dr=2.0, r_max=14.0)
    c = np.array([[20, 21, 19]])
    x = W.paint_bubbles(n, c + 0.5, [rb], x_in=1.0)
    r = orc.max_radius(mp, n, True, x, c)[0]
    h = math.sqrt(3) / 2
    assert rb - h - mp.dr < r <= rb + h
    assert r == 2.0 * math.floor(r / 2.0)


def test_max_radius_limits(orc):
    n = 24
    mp = orc.make_merge_params(dr=2.0, r_max=8.0)
    c = np.array([[5, 5, 5], [12, 3, 20]])
    assert list(orc.max_radius(mp, n, True, np.ones((n, n, n)), c)) == [8.0, 8.0]
    assert list(orc.max_radius(mp, n, True, np.zeros((n, n, n)), c)) == [0.0, 0.0]
    # non-periodic box near a corner: samples outside the box are dropped
    assert orc.max_radius(mp, n, False, np.ones((n, n, n)), np.array([[0, 0, 0]]))[0] == 8.0


def _bfs_groups(cells, rad, n, periodic, mp):
    m = len(cells)
    adj = [[] for _ in range(m)]
    for a in range(m):
        for b in range(a + 1, m):
            if not (rad[a] > 0 and rad[b] > 0):
                continue
            d = cells[a].astype(np.int64) - cells[b]
            if periodic:
                d = np.mod(d, n)
                d = np.where(2 * d > n, d - n, d)
            rs = mp.f_ov * (rad[a] + rad[b])
            if float((d * d).sum()) <= rs * rs + mp.eps:
                adj[a].append(b)
                adj[b].append(a)
    seen, groups = [False] * m, []
    for a in range(m):
        if seen[a]:
            continue
        q, comp = deque([a]), []
        seen[a] = True
        while q:
            u = q.popleft()
            comp.append(u)
            for v in adj[u]:
                if not seen[v]:
                    seen[v] = True
                    q.append(v)
        groups.append(sorted(comp))
    return groups


@pytest.mark.parametrize("n,periodic,seed", [(40, True, 1), (40, False, 2), (64, True, 3)])
def test_merge_groups_against_bfs(orc, n, periodic, seed):
    """n = 64 with R_max = 8 exercises the oracle's binned pair search."""
    g = np.random.default_rng(seed)
    mp = orc.make_merge_params(dr=2.0, r_max=8.0)
    pos, centres = W.clustered_cells(n, 12, 20, 2.0, g)
    ndot = W.lognormal_values(len(pos), 1e50, 2.0, g)
    x = W.paint_bubbles(n, centres[:8], g.uniform(3, 9, 8), periodic=periodic)
    cells, flux = orc.dedupe_sort(n, pos, ndot)
    rad = orc.max_radius(mp, n, periodic, x, cells)
    groups = _bfs_groups(cells, rad, n, periodic, mp)
    assert any(len(gr) > 1 for gr in groups)
    mc, mf, mr = orc.merge_sources(mp, n, periodic, x, pos, ndot)
    assert len(mc) == len(groups)
    keys = [tuple(c) for c in mc]
    assert keys == sorted(keys)
    assert mf.sum() == pytest.approx(ndot.sum(), rel=1e-13)
    by_cell = {tuple(c): (f, r) for c, f, r in zip(mc, mf, mr)}
    for gr in groups:
        members = {tuple(cells[k]) for k in gr}
        hit = [c for c in members if c in by_cell]
        assert len(hit) == 1  # the merged source sits on exactly one member cell
        f, r = by_cell[hit[0]]
        assert f == pytest.approx(flux[gr].sum(), rel=1e-13)
        assert r == rad[gr].max()


def test_merge_centroid_snap_exact(orc):
    """Flux-weighted centroid, rounded, snapped to the nearest member cell;
    the second case unwraps across the periodic edge."""
    n = 32
    mp = orc.make_merge_params(dr=2.0, r_max=8.0, n_min=1)
    x = np.ones((n, n, n))
    # (10 + 11 + 6*14) / 8 = 13.125 -> 13 -> nearest member x = 14
    pos = np.array([[10.5, 10.5, 10.5], [11.5, 10.5, 10.5], [14.5, 10.5, 10.5]])
    mc, mf, _ = orc.merge_sources(mp, n, True, x, pos, [1.0, 1.0, 6.0])
    np.testing.assert_array_equal(mc, [[14, 10, 10]])
    assert mf[0] == 8.0
    # members at x = 1 and x = n - 2 (3 cells apart through the edge):
    # unwrapped relative to x = 1: {1, -2}; (1 + 3 * -2) / 4 = -1.25 -> -1 -> n - 1;
    # nearest member is n - 2
    pos = np.array([[1.5, 5.5, 5.5], [n - 1.5, 5.5, 5.5]])
    mc, mf, _ = orc.merge_sources(mp, n, True, x, pos, [1.0, 3.0])
    np.testing.assert_array_equal(mc, [[n - 2, 5, 5]])
    # without periodic wrap the two are far apart and stay separate
    mc, _, _ = orc.merge_sources(mp, n, False, x, pos, [1.0, 3.0])
    assert len(mc) == 2


def test_max_radius_few_samples_need_all_ionized(orc):
    """When a shell holds fewer than N_min distinct sample cells, every one
    must be ionized (Alg. source_merge).  With the 12 level-0 directions the
    first shell has at most 12 samples: a single neutral sample cell then
    stops the growth at 0 under N_min = 20, but not under N_min = 1 with
    f_req = 0.9 when 11 of 12 samples are ionized."""
    n = 24
    c = np.array([[12, 12, 12]])
    x = np.ones((n, n, n))
    d = orc.pix2vec_nest(0, 4)  # the +x equatorial direction
    p = np.floor(c[0] + 0.5 + 2.0 * d).astype(int)
    x[p[2], p[1], p[0]] = 0.0  # that sample cell is neutral
    mp = orc.make_merge_params(dr=2.0, r_max=6.0, n_min=20, shell_level=0, f_req=0.9)
    assert orc.max_radius(mp, n, True, x, c)[0] == 0.0
    mp = orc.make_merge_params(dr=2.0, r_max=2.0, n_min=1, shell_level=0, f_req=0.9)
    assert orc.max_radius(mp, n, True, x, c)[0] == 2.0  # 11/12 >= 0.9
    mp = orc.make_merge_params(dr=2.0, r_max=2.0, n_min=1, shell_level=0, f_req=0.95)
    assert orc.max_radius(mp, n, True, x, c)[0] == 0.0  # 11/12 < 0.95
