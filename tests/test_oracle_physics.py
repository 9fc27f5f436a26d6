"""Pins for the oracle's deposit, correction, splitting and budget.

Closed forms and invariants that the paper's definitions fix:
  * Beer-Lambert attenuation along one ray and the per-cell absorbed photon
    rate L e^{-tau_in} (1 - e^{-dtau}) that Eq. lut_eqn deposits;
  * the optically thin limit (footnote in Sec. "Numerical instability for low
    n_H neighbor cells"): Gamma = L sigma0 dl / h^3 per segment, and the
    1/r^2 flux sigma0 Ndot / (4 pi r^2) of a point source;
  * photon conservation: emitted = absorbed + escaped + truncated, and
    sum_c Gamma_c a_c h^3 = absorbed under the conservative correction
    (Eqs. new_correction / new_secondary), lossy under Eq. correction alone;
  * the correction moves deposits only (A, X, T do not depend on it), and
    its value for a ray through cell centres (Eq. correction, Eq.
    secondary_correction);
  * superposition over sources and linearity in Ndot;
  * the split tree of Eq. split_criterion: 12 * 4^l rays at level l while
    every level-(l-1) ray reaches its split radius.
"""
import math

import numpy as np
import pytest

import workloads as W
from bruteforce import box_exit, cells_along

SIG = 6.30e-18


def _uniform(n, nH=1e-3, x=0.0):
    return np.full((n, n, n), nH), np.full((n, n, n), x)


def test_beer_lambert_single_ray(orc):
    n, h = 10, 1.0e20
    nH, x = _uniform(n, 2e-3, 0.25)
    a = 2e-3 * 0.75
    p = orc.make_params(n, h, periodic=False, n_min_ray=0.0, corr=orc.CORR_NONE)
    g = np.random.default_rng(5)
    for _ in range(10):
        o = g.random(3) * n
        d = g.standard_normal(3)
        d /= np.linalg.norm(d)
        L = 3.7e45
        gamma, b, _ = orc.trace_rays(p, nH, x, o[None], d[None], 0, L)
        s_exit = box_exit(o, d, n)
        k = SIG * a * h  # optical depth per cell length
        assert b["escaped"] == pytest.approx(L * math.exp(-k * s_exit), rel=1e-13)
        assert b["absorbed"] == pytest.approx(L * -math.expm1(-k * s_exit), rel=1e-13)
        # per-cell photons from the brute-force geometry
        expect = np.zeros((n, n, n))
        for (i, j, kk), t0, t1 in cells_along(o, d, 0.0, s_exit):
            expect[kk, j, i] += L * math.exp(-k * t0) * -math.expm1(-k * (t1 - t0))
        np.testing.assert_allclose(gamma * a * h ** 3, expect, rtol=1e-12, atol=1e-14 * L)


def test_thin_limit_and_fully_ionized(orc):
    """x = 1: no absorption, Gamma = L sigma0 dl / h^3 per segment, all escape."""
    n, h = 8, 3.0e19
    nH, x = _uniform(n, 1e-3, 1.0)
    p = orc.make_params(n, h, periodic=False, n_min_ray=0.0, corr=orc.CORR_CONSERVATIVE)
    o = np.array([1.3, 2.2, 0.4])
    d = np.array([0.3, 0.5, 0.8])
    d /= np.linalg.norm(d)
    L = 1e40
    gamma, b, _ = orc.trace_rays(p, nH, x, o[None], d[None], 2, L)
    assert b["absorbed"] == 0.0 and b["escaped"] == L
    expect = np.zeros((n, n, n))
    for (i, j, k), t0, t1 in cells_along(o, d, 0.0, box_exit(o, d, n)):
        expect[k, j, i] += L * SIG * (t1 - t0) * h / h ** 3
    np.testing.assert_allclose(gamma, expect, rtol=1e-12, atol=1e-12 * expect.max())


def test_correction_through_cell_centres(orc):
    """A ray along +x through cell centres: each segment's midpoint is
    D_edge = 1/2 from every face (after the first), the tie goes to the +x
    face, so Eq. correction gives f_c = 1/2 + 1/(2 L_pix) with L_pix = r_m
    sqrt(Omega(0)) once L_pix > 1, and Eq. secondary_correction puts
    (1 - f_c) G a_c / a_{c+1} into the next cell."""
    n, h = 12, 2.0e19
    g = np.random.default_rng(3)
    nH = np.full((n, n, n), 1e-3)
    nH[1, 1, :] = 1e-3 * (0.5 + g.random(n))  # density varies along the ray
    x = np.zeros((n, n, n))
    p = orc.make_params(n, h, periodic=False, n_min_ray=0.0, n_th=0.0,
                        corr=orc.CORR_CONSERVATIVE)
    o = np.array([0.5, 1.5, 1.5])
    L = 1e44
    gamma, b, _ = orc.trace_rays(p, nH, x, o[None], np.array([[1.0, 0.0, 0.0]]), 0, L)
    a = nH[1, 1, :]
    sq = math.sqrt(4 * math.pi / 12)
    expect = np.zeros(n)
    tau = 0.0
    for i in range(n):
        s0 = 0.0 if i == 0 else i - 0.5
        s1 = i + 0.5
        ds = s1 - s0
        dtau = SIG * a[i] * ds * h
        G = L * math.exp(-tau) * -math.expm1(-dtau) / (a[i] * h ** 3)
        rm = 0.5 * (s0 + s1)
        lpix = rm * sq
        dedge = 0.25 if i == 0 else 0.5
        if i + 1 < n and dedge < 0.5 * lpix:
            fc = 0.5 + dedge / lpix
            expect[i] += fc * G
            expect[i + 1] += (1 - fc) * G * a[i] / a[i + 1]
        else:
            expect[i] += G
        tau += dtau
    np.testing.assert_allclose(gamma[1, 1, :], expect, rtol=1e-12)
    assert np.count_nonzero(gamma) == np.count_nonzero(expect)


def _field_case(n=24, seed=11, periodic=True):
    g = np.random.default_rng(seed)
    nH = W.lognormal_density(n, 1e-3, 1.0, g)
    x = np.where(g.random((n, n, n)) < 0.3, 1.0 - 1e-4, 0.0)
    x[g.random((n, n, n)) < 0.05] = 1.0  # some fully ionized cells
    pos = g.random((5, 3)) * n
    ndot = W.lognormal_values(5, 1e50, 1.0, g)
    h = 0.3 / (SIG * 1e-3)
    return n, h, nH, x, pos, ndot, periodic


@pytest.mark.parametrize("periodic", [True, False])
@pytest.mark.parametrize("corr", [0, 1, 2, 3, 4])
def test_budget_identity_and_correction_invariance(orc, periodic, corr):
    n, h, nH, x, pos, ndot, _ = _field_case(periodic=periodic)
    base = orc.make_params(n, h, periodic=periodic, n_min_ray=4.0, l_max=6, tau_max=12.0,
                           n_th=3e-4, corr=orc.CORR_NONE)
    p = orc.make_params(n, h, periodic=periodic, n_min_ray=4.0, l_max=6, tau_max=12.0,
                        n_th=3e-4, corr=corr)
    g0, b0 = orc.trace(base, nH, x, pos, ndot)
    g1, b1 = orc.trace(p, nH, x, pos, ndot)
    E = b1["emitted"]
    assert abs(E - b1["absorbed"] - b1["escaped"] - b1["truncated"]) <= 1e-12 * E
    for k in ("absorbed", "escaped", "truncated"):
        assert b1[k] == pytest.approx(b0[k], rel=1e-12, abs=1e-12 * E)
    for k in ("segments", "rays", "splits", "rays_per_level"):
        assert b1[k] == b0[k]
    a = (1 - x) * nH
    deposited = (g1 * a * h ** 3).sum()
    if corr in (orc.CORR_NONE, orc.CORR_CONSERVATIVE):
        assert deposited == pytest.approx(b1["absorbed"], rel=1e-12)
    else:
        assert deposited < b1["absorbed"] * (1 - 1e-6)  # photons lost
    if corr != orc.CORR_NONE:
        assert np.abs(g1 - g0).max() > 1e-3 * g0.max()


def test_superposition_and_linearity(orc):
    n, h, nH, x, pos, ndot, periodic = _field_case(seed=21)
    p = orc.make_params(n, h, periodic=True, n_min_ray=4.0, l_max=6, tau_max=20.0, n_th=3e-4)
    gall, ball = orc.trace(p, nH, x, pos, ndot)
    parts = [orc.trace(p, nH, x, pos[k:k + 1], ndot[k:k + 1]) for k in range(len(ndot))]
    gsum = sum(g for g, _ in parts)
    np.testing.assert_allclose(gall, gsum, rtol=0, atol=1e-12 * gall.max())
    assert ball["segments"] == sum(b["segments"] for _, b in parts)
    g3, _ = orc.trace(p, nH, x, pos, 3.0 * ndot)
    np.testing.assert_allclose(g3, 3.0 * gall, rtol=1e-12, atol=1e-13 * gall.max())


def test_split_tree_counts(orc):
    """Thin uniform open box, source at the centre of cell (32,32,32) of a
    64^3 grid: the nearest face is 31.5 cells away.  A ray is tested for a
    split at cell boundaries inside the box, so every level-(l-1) ray splits
    when R_split(l-1) + sqrt(3) (the longest cell chord) is below 31.5, with
    R_split(l) = 1/sqrt(N_min Omega(l)).  That holds up to l-1 = 5, so levels
    0..6 hold exactly 12 * 4^l rays; R_split(7) = 62.5 exceeds the corner
    distance 31.5 sqrt(3) + sqrt(3), so no ray reaches level 8."""
    n = 64
    h = 1e-6 / (SIG * 1e-3)  # tau per cell = 1e-6
    nH, x = _uniform(n)
    p = orc.make_params(n, h, periodic=False, n_min_ray=4.0, l_max=9, tau_max=30.0)
    _, b = orc.trace(p, nH, x, [[32.5, 32.5, 32.5]], [1e50])
    r = [1.0 / math.sqrt(4.0 * 4 * math.pi / (12 * 4 ** l)) for l in range(10)]
    assert r[5] + math.sqrt(3) < 31.5 < r[6] + math.sqrt(3)
    assert r[7] > (31.5 + 1) * math.sqrt(3)
    assert b["rays_per_level"][:7] == [12 * 4 ** l for l in range(7)]
    assert 0 < b["rays_per_level"][7] < 12 * 4 ** 7
    assert b["rays_per_level"][8] == 0
    assert b["splits"] == sum(12 * 4 ** l for l in range(6)) + b["rays_per_level"][7] // 4
    assert b["truncated"] == 0.0


def test_inverse_square_thin_medium(orc):
    """Shell-averaged Gamma in an optically thin open box against the exact
    sigma0 Ndot e^{-tau} / (4 pi r^2 h^2) of a point source (2 %)."""
    n = 64
    h = 1e-6 / (SIG * 1e-3)
    nH, x = _uniform(n)
    p = orc.make_params(n, h, periodic=False, n_min_ray=4.0, l_max=9, tau_max=30.0,
                        n_th=0.0, corr=orc.CORR_CONSERVATIVE)
    src = np.array([32.5, 32.5, 32.5])
    Nd = 1e50
    gamma, b = orc.trace(p, nH, x, src[None], [Nd])
    c = np.arange(n) + 0.5
    r = np.sqrt((c[None, None, :] - src[0]) ** 2 + (c[None, :, None] - src[1]) ** 2 +
                (c[:, None, None] - src[2]) ** 2)
    with np.errstate(divide="ignore"):
        exact = SIG * Nd * np.exp(-1e-6 * r) / (4 * np.pi * (r * h) ** 2)
    for r0 in range(4, n // 2 - 2):
        sel = (r >= r0) & (r < r0 + 1)
        assert gamma[sel].mean() / exact[sel].mean() == pytest.approx(1.0, abs=0.02), r0
    a = (1 - x) * nH
    assert (gamma * a * h ** 3).sum() == pytest.approx(b["absorbed"], rel=1e-12)


def test_correction_variant_identities(orc):
    """Exact consequences of the definitions, on a field where every cell
    keeps some neutral gas (a > 0): naive thresholding with n_th = 0 is the
    conservative scheme (every neighbour is usable, so both apply f_c and
    deposit the neighbour share); with a threshold above every density no
    neighbour is usable, so naive thresholding is Eq. correction alone
    (LINEAR) and the conservative scheme deposits everything in the cell
    (NONE); squaring f_c <= 1 loses more photons than LINEAR."""
    n, h, nH, x, pos, ndot, _ = _field_case(seed=33)
    x = np.minimum(x, 1.0 - 1e-4)
    kw = dict(periodic=True, n_min_ray=4.0, l_max=6, tau_max=20.0)
    run = lambda corr, n_th: orc.trace(orc.make_params(n, h, corr=corr, n_th=n_th, **kw),
                                       nH, x, pos, ndot, nthreads=1)  # one summation order
    g_naive0, _ = run(orc.CORR_NAIVE, 0.0)
    g_cons0, _ = run(orc.CORR_CONSERVATIVE, 0.0)
    np.testing.assert_array_equal(g_naive0, g_cons0)
    big = 10.0 * nH.max()
    g_naive_big, _ = run(orc.CORR_NAIVE, big)
    g_lin, b_lin = run(orc.CORR_LINEAR, big)
    np.testing.assert_array_equal(g_naive_big, g_lin)
    g_cons_big, b = run(orc.CORR_CONSERVATIVE, big)
    g_none, _ = run(orc.CORR_NONE, big)
    np.testing.assert_array_equal(g_cons_big, g_none)  # nothing usable: f_c = 1 everywhere
    g_sq, _ = run(orc.CORR_SQUARED, big)
    a = (1 - x) * nH
    dep = lambda g: (g * a * h ** 3).sum()
    assert dep(g_sq) < dep(g_lin) < b_lin["absorbed"]


def test_tau_max_stop_at_the_boundary(orc):
    """Alg. functors, ray_fltr: a monochromatic ray stops at the first cell
    boundary where its optical depth reaches tau_max (tested before the
    advance, >= not >), and its remaining photons L e^{-tau} are booked as
    truncated, not escaped.  One ray along +x from the plane x = 0 through a
    uniform open box with sigma0 = h = 1 and a = 1/2, so that every cell adds
    exactly dtau = 1/2 and the optical depth at boundary k is exactly k/2:
    the ray stops after k = min{k : k/2 >= tau_max} segments."""
    n = 64
    nH, x = np.full((n, n, n), 0.5), np.zeros((n, n, n))
    L = 1e48
    for tau_max, k in ((3.0, 6), (2.7, 6), (3.2, 7), (0.5, 1), (0.4, 1)):
        p = orc.make_params(n, 1.0, periodic=False, sigma0=1.0, n_min_ray=0.0,
                            corr=orc.CORR_NONE, tau_max=tau_max)
        gamma, b, log = orc.trace_rays(p, nH, x, np.array([[0.0, 32.5, 32.5]]),
                                       np.array([[1.0, 0.0, 0.0]]), 0, L, max_log=n)
        assert b["segments"] == k, tau_max
        assert [tuple(v) for v in log["ijk"]] == [(c, 32, 32) for c in range(k)]
        assert b["escaped"] == 0.0
        assert b["truncated"] == pytest.approx(L * math.exp(-0.5 * k), rel=1e-14)
        assert b["absorbed"] == pytest.approx(L * -math.expm1(-0.5 * k), rel=1e-14)
        # cell c absorbs L e^{-c/2} (1 - e^{-1/2}); Gamma = dN / (a h^3)
        expect = L * np.exp(-0.5 * np.arange(k)) * -math.expm1(-0.5) / 0.5
        np.testing.assert_allclose(gamma[32, 32, :k], expect, rtol=1e-14)
        assert np.count_nonzero(gamma) == k


def _first_crossing_beyond(o, d, r):
    """Smallest plane crossing t = (plane - o_a) / d_a of the line o + t d
    with t^2 > r^2 (the cell boundary where a ray first needs to split)."""
    best = math.inf
    for a in range(3):
        if d[a] == 0.0:
            continue
        # planes between o_a and o_a + (r + 2) d_a, on the side the ray travels
        lo = math.floor(min(o[a], o[a] + (r + 2) * d[a])) - 1
        hi = math.ceil(max(o[a], o[a] + (r + 2) * d[a])) + 1
        for plane in range(lo, hi + 1):
            t = (plane - o[a]) / d[a]
            if t > 0 and t * t > r * r:
                best = min(best, t)
    return best


def test_l_max_truncates_rays_that_need_to_split(orc):
    """Alg. functors, ray_fltr with the reading that a ray at level l_max
    marches until it would need to split and is then terminated into the
    truncated term.  In the thin uniform open box of test_split_tree_counts
    every ray up to level 5 reaches its split radius inside the box, so with
    l_max = 4 levels 0..4 hold exactly 12 * 4^l rays, no ray reaches level
    5, and each of the 3072 level-4 rays carries Ndot / 3072 and stops at the
    first cell boundary s beyond its split radius R_split(4), with optical
    depth kappa s (kappa = sigma0 a h per cell)."""
    n = 64
    kappa = 1e-3
    h = kappa / (SIG * 1e-3)
    nH, x = _uniform(n)
    src = np.array([32.5, 32.5, 32.5])
    Nd = 1e50
    lmax = 4
    p = orc.make_params(n, h, periodic=False, n_min_ray=4.0, l_max=lmax, tau_max=30.0)
    gamma, b = orc.trace(p, nH, x, src[None], [Nd])
    assert b["rays_per_level"][:lmax + 1] == [12 * 4 ** l for l in range(lmax + 1)]
    assert b["rays_per_level"][lmax + 1:] == [0] * (len(b["rays_per_level"]) - lmax - 1)
    assert b["splits"] == sum(12 * 4 ** l for l in range(lmax))
    r4 = 1.0 / math.sqrt(4.0 * 4 * math.pi / (12 * 4 ** lmax))
    assert r4 + math.sqrt(3) < 31.5
    dirs = orc.healpix_dirs(lmax)
    s_stop = np.array([_first_crossing_beyond(src, d, r4) for d in dirs])
    assert np.all((s_stop > r4) & (s_stop <= r4 + math.sqrt(3)))
    expect_T = (Nd / (12 * 4 ** lmax)) * np.exp(-kappa * s_stop).sum()
    assert b["truncated"] == pytest.approx(expect_T, rel=1e-12)
    assert b["escaped"] == 0.0
    assert b["absorbed"] == pytest.approx(Nd - expect_T, rel=1e-12)
    # nothing is deposited beyond the level-4 stop radius
    c = np.arange(n) + 0.5
    r = np.sqrt((c[None, None, :] - src[0]) ** 2 + (c[None, :, None] - src[1]) ** 2 +
                (c[:, None, None] - src[2]) ** 2)
    assert gamma[r > s_stop.max() + math.sqrt(3)].max() == 0.0
    assert gamma[r < r4 - math.sqrt(3)].min() > 0.0
