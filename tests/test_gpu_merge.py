"""GPU source merging (Sec. "Source Merging Algorithm", Alg. source_merge)
against the oracle, through the C ABI.  The catalogue is integer work
(cells, radii, group membership) and must match exactly; merged rates are
sums taken in the same order on both sides and must match to 1e-13."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def gpu_merge(gpu, n, periodic, x, pos, ndot, mp):
    ctx = gpu.init_grid(gpu.make_desc(n, 1e21, periodic=periodic), np.full((n, n, n), 1e-4), x,
                        device="cuda:0", max_sources=len(ndot), ray_capacity=4096)
    ctx.add_sources(pos, ndot)
    m2 = ctx.merge_sources(mp)
    p, f, r = ctx.get_sources()
    ctx.destroy()
    assert len(f) == m2
    return p, f, r


def check_same(orc_out, gpu_out):
    oc, of, orr = orc_out
    gp, gf, gr = gpu_out
    assert len(gf) == len(of)
    np.testing.assert_array_equal(np.floor(gp).astype(np.int32), oc)
    np.testing.assert_array_equal(gp - np.floor(gp), 0.5)  # cell centres
    np.testing.assert_array_equal(gr, orr)
    np.testing.assert_allclose(gf, of, rtol=1e-13, atol=0)


@pytest.mark.parametrize("n,periodic,seed,r_max", [(40, True, 1, 8.0), (40, False, 2, 8.0),
                                                   (64, True, 3, 8.0), (96, True, 4, 6.0),
                                                   (96, False, 5, 6.0)])
def test_merge_matches_oracle(gpu, orc, n, periodic, seed, r_max):
    g = np.random.default_rng(seed)
    pos, centres = W.clustered_cells(n, 16, 24, 2.0, g)
    pos[:40] = W.uniform_positions(40, n, g)  # some continuous positions too
    ndot = W.lognormal_values(len(pos), 1e50, 2.0, g)
    x = W.paint_bubbles(n, centres[:10], g.uniform(3, 12, 10), periodic=periodic)
    x[g.random((n, n, n)) < 0.02] = 0.95  # scattered ionized cells
    kw = dict(dr=2.0, r_max=r_max)
    ref = orc.merge_sources(orc.make_merge_params(**kw), n, periodic, x, pos, ndot)
    got = gpu_merge(gpu, n, periodic, x, pos, ndot, gpu.make_merge_params(**kw))
    assert len(ref[1]) < len(np.unique(np.floor(pos), axis=0))  # something merged
    check_same(ref, got)


def test_merge_degenerate(gpu, orc):
    n = 16
    x = np.ones((n, n, n))
    mp_o, mp_g = orc.make_merge_params(), gpu.make_merge_params()
    # all sources in one cell
    pos = np.full((7, 3), 5.25) + np.linspace(0, 0.5, 7)[:, None]
    ndot = np.arange(1.0, 8.0)
    check_same(orc.merge_sources(mp_o, n, True, x, pos, ndot),
               gpu_merge(gpu, n, True, x, pos, ndot, mp_g))
    # nothing ionized: dedupe and sort only
    g = np.random.default_rng(9)
    pos = W.uniform_positions(50, n, g)
    ndot = g.random(50)
    z = np.zeros((n, n, n))
    ref = orc.merge_sources(mp_o, n, True, z, pos, ndot)
    check_same(ref, gpu_merge(gpu, n, True, z, pos, ndot, mp_g))
    assert (ref[2] == 0).all()
    # a single source, and an ionized box where everything merges
    check_same(orc.merge_sources(mp_o, n, True, x, pos[:1], ndot[:1]),
               gpu_merge(gpu, n, True, x, pos[:1], ndot[:1], mp_g))
    ref = orc.merge_sources(mp_o, n, True, x, pos, ndot)
    assert len(ref[1]) == 1
    check_same(ref, gpu_merge(gpu, n, True, x, pos, ndot, mp_g))


@pytest.mark.slow
def test_merge_clustered_512(gpu, orc):
    """The 512^3 clustered catalogue at full size: 512 clusters x 64 sources
    (sigma 2 cells), 200 bubbles r ~ U[4, 20] on cluster centres."""
    n = 512
    pos, centres = W.clustered_cells(n, 512, 64, 2.0, W.rng(4, 1))
    ndot = W.lognormal_values(pos.shape[0], 1e50, 2.0, W.rng(4, 2))
    g = W.rng(4, 3)
    pick = g.choice(512, size=200, replace=False)
    x = W.paint_bubbles(n, centres[pick], g.uniform(4.0, 20.0, size=200))
    ref = orc.merge_sources(orc.make_merge_params(), n, True, x, pos, ndot)
    got = gpu_merge(gpu, n, True, x, pos, ndot, gpu.make_merge_params())
    assert len(ref[1]) < 0.9 * len(ndot)
    check_same(ref, got)


def test_trace_after_merge(gpu, orc):
    """Trace the merged catalogue on the GPU and in the oracle (which traces
    its own merged catalogue): same sources, same Gamma."""
    n = 32
    g = np.random.default_rng(17)
    pos, centres = W.clustered_cells(n, 6, 20, 2.0, g)
    ndot = W.lognormal_values(len(pos), 1e50, 2.0, g)
    x = W.paint_bubbles(n, centres[:4], g.uniform(4, 8, 4))
    nH = W.lognormal_density(n, 1e-3, 1.0, g)
    h = 0.5 / (W.SIGMA0 * 1e-3)
    kw = dict(periodic=True, n_min_ray=4.0, l_max=6, tau_max=30.0, n_th=1e-5)
    mc, mf, _ = orc.merge_sources(orc.make_merge_params(), n, True, x, pos, ndot)
    ref, rb = orc.trace(orc.make_params(n, h, **kw), nH, x, mc + 0.5, mf)
    ctx = gpu.init_grid(gpu.make_desc(n, h, **kw), nH, x, device="cuda:0",
                        max_sources=len(ndot), ray_capacity=1 << 18)
    ctx.add_sources(pos, ndot)
    assert ctx.merge_sources(gpu.make_merge_params()) == len(mf)
    gamma, b = ctx.trace_step()
    ctx.destroy()
    got = gamma.cpu().numpy()
    mask = ref > 1e-6 * ref.max()
    assert np.abs(got[mask] / ref[mask] - 1).max() <= 1e-10
    assert b["segments"] == rb["segments"]
