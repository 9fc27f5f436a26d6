"""GPU parity of the ray-tracing sweep against the oracle, through the C ABI.

Bars (stated in the build's target): on cells with Gamma > 1e-6 max Gamma,
the FP64 path matches the oracle to relative error 1e-10 and the mixed path
to 1e-4; photon-budget terms match to 1e-6 of the emitted rate (FP64: 1e-10).
Segment, ray and split counts are integers decided in FP64 on both sides and
must be equal, in both precisions: the mixed path accumulates the optical
depth that its tau_max stop reads in FP64 from the FP64 absorber, by the
same operations as the FP64 path, so it takes the same decisions.
"""
import math

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def rel_err(got, ref, floor=1e-6):
    got, ref = np.asarray(got), np.asarray(ref)
    mask = ref > floor * ref.max()
    e_in = np.abs(got[mask] / ref[mask] - 1).max() if mask.any() else 0.0
    e_out = np.abs(got[~mask] - ref[~mask]).max() / ref.max() if (~mask).any() else 0.0
    return e_in, e_out


def budget_err(b, rb):
    E = rb["emitted"]
    return max(abs(b[k] - rb[k]) for k in ("absorbed", "escaped", "truncated")) / E


def field_case(n, seed, ionized=0.3, m=5, mean=1e-3, tau_cell=0.5):
    g = np.random.default_rng(seed)
    nH = W.lognormal_density(n, mean, 1.0, g)
    x = np.where(g.random((n, n, n)) < ionized, 1.0 - 1e-4, 0.0)
    x[g.random((n, n, n)) < 0.03] = 1.0
    pos = W.uniform_positions(m, n, g)
    ndot = W.lognormal_values(m, 1e50, 1.0, g)
    h = tau_cell / (W.SIGMA0 * mean)
    return nH, x, pos, ndot, h


def run_gpu(gpu, n, h, nH, x, pos, ndot, prec, cap=1 << 18, **kw):
    ctx = gpu.init_grid(gpu.make_desc(n, h, precision=prec, **kw), nH, x, device="cuda:0",
                        max_sources=max(len(ndot), 1), ray_capacity=cap)
    ctx.add_sources(pos, ndot)
    gamma, b = ctx.trace_step()
    out = gamma.cpu().numpy()
    ctx.destroy()
    return out, b


BENCH_CAPACITY = 1 << 25  # ray slots per level queue in bench.py


def run_gpu_replayed(gpu, w, prec, pos=None, ndot=None, merge=False):
    """The workload as bench.py times it: 2^25-slot level queues, the launch
    parameters bench.py sets for it, one eager pass, then the captured
    device-driven pass replayed; returns the replayed pass's Gamma and budget
    (and the traced catalogue when merging)."""
    import bench
    pos = w.pos if pos is None else pos
    ndot = w.ndot if ndot is None else ndot
    desc = gpu.make_desc(w.n, w.h_cm, precision=prec, periodic=w.periodic, n_min_ray=w.n_min_ray,
                         l_max=w.l_max, tau_max=w.tau_max, n_th=w.n_th)
    ctx = gpu.init_grid(desc, w.n_H, w.x, device="cuda:0", max_sources=len(ndot),
                        ray_capacity=BENCH_CAPACITY)
    refill, claim = bench.launch_params(w.name) or (0, 0)
    ctx.set_tuning(refill_min=refill, claim=claim)
    ctx.add_sources(pos, ndot)
    cat = None
    if merge:
        ctx.merge_sources(gpu.make_merge_params())
        cat = ctx.get_sources()
    g, _ = ctx.trace_step()
    g, b = ctx.trace_step(g)
    assert ctx.last_pass_was_graph()
    out = g.cpu().numpy()
    ctx.destroy()
    return out, b, cat


def test_device_healpix_matches_oracle(gpu, orc):
    """The march's directions: the table levels (built on the host with the C
    library's cos and sin) equal the oracle's bit for bit, so the FP64 paths
    take their decisions on the same directions; levels past the table come
    from the device's cos and sin, within an ulp of the oracle's."""
    n = 4
    ctx = gpu.init_grid(gpu.make_desc(n, 1e20, l_max=7), np.ones((n, n, n)),
                        np.zeros((n, n, n)), device="cuda:0", max_sources=1, ray_capacity=4096)
    for level in range(0, 8):
        dev = ctx.healpix_dirs(level)
        np.testing.assert_array_equal(dev, orc.healpix_dirs(level), err_msg=str(level))
    for level in (8, 10, 14):  # past the table: the device function
        npix = 12 * 4 ** level
        first = [0, npix // 3, npix - 64]
        for f in first:
            dev = ctx.healpix_dirs(level, f, 64)
            ref = np.array([orc.pix2vec_nest(level, p) for p in range(f, f + 64)])
            assert np.abs(dev - ref).max() <= 4.5e-16, (level, f)
            np.testing.assert_array_equal(dev[:, 2], ref[:, 2])  # z is exact on both sides
    ctx.destroy()


@pytest.mark.parametrize("periodic", [False, True])
@pytest.mark.parametrize("prec", [0, 1])
def test_injected_rays(gpu, orc, periodic, prec):
    n, h = 12, 3.0e19
    g = np.random.default_rng(40 + periodic)
    nH = W.lognormal_density(n, 1e-3, 1.0, g)
    x = np.where(g.random((n, n, n)) < 0.3, 1.0, 0.0)
    k = 300
    o = g.random((k, 3)) * n
    d = g.standard_normal((k, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    lev = g.integers(0, 6, k).astype(np.int32)
    L = 10 ** g.uniform(40, 45, k)
    kw = dict(periodic=periodic, n_min_ray=0.0, l_max=7, tau_max=30.0, n_th=4e-4)
    ref, rb, _ = orc.trace_rays(orc.make_params(n, h, **kw), nH, x, o, d, lev, L)
    ctx = gpu.init_grid(gpu.make_desc(n, h, precision=prec, **kw), nH, x, device="cuda:0",
                        max_sources=1, ray_capacity=4096)
    gamma, b = ctx.trace_rays_debug(o, d, lev, L)
    ctx.destroy()
    e_in, e_out = rel_err(gamma.cpu().numpy(), ref)
    tol = 1e-12 if prec == 0 else 1e-4
    assert e_in <= tol and e_out <= tol
    assert b["segments"] == rb["segments"]
    assert budget_err(b, rb) <= (1e-13 if prec == 0 else 1e-6)


@pytest.mark.parametrize("periodic", [True, False])
@pytest.mark.parametrize("corr", [0, 1, 2, 3, 4])
def test_trace_fp64_matches_oracle(gpu, orc, periodic, corr):
    n = 24
    nH, x, pos, ndot, h = field_case(n, 100 + corr + 10 * periodic)
    kw = dict(periodic=periodic, n_min_ray=4.0, l_max=6, tau_max=25.0, n_th=4e-4, corr=corr)
    ref, rb = orc.trace(orc.make_params(n, h, **kw), nH, x, pos, ndot)
    got, b = run_gpu(gpu, n, h, nH, x, pos, ndot, 0, **kw)
    e_in, e_out = rel_err(got, ref)
    assert e_in <= 1e-10 and e_out <= 1e-10, (e_in, e_out)
    for k in ("segments", "rays", "splits"):
        assert b[k] == rb[k], k
    assert b["rays_per_level"] == rb["rays_per_level"][:15]
    assert budget_err(b, rb) <= 1e-10
    assert b["emitted"] == rb["emitted"]


COUNTS = ("segments", "rays", "splits", "rays_per_level")


def same_counts(b, rb):
    for k in COUNTS:
        ref = rb[k][:15] if k == "rays_per_level" else rb[k]
        assert b[k] == ref, (k, b[k], ref)


@pytest.mark.parametrize("n,periodic", [(13, True), (31, False), (33, True)])
def test_odd_grids_match_oracle(gpu, orc, n, periodic):
    """Grids whose cell count is not a multiple of the 8-cell Gamma line (the
    last line of the LDS deposit table reaches past the grid): both paths
    against the oracle."""
    nH, x, pos, ndot, h = field_case(n, 300 + n, m=4)
    kw = dict(periodic=periodic, n_min_ray=4.0, l_max=7, tau_max=25.0, n_th=4e-4)
    ref, rb = orc.trace(orc.make_params(n, h, **kw), nH, x, pos, ndot)
    got, b = run_gpu(gpu, n, h, nH, x, pos, ndot, 0, **kw)
    assert rel_err(got, ref)[0] <= 1e-10
    assert b["segments"] == rb["segments"] and b["splits"] == rb["splits"]
    assert budget_err(b, rb) <= 1e-10
    gm, bm = run_gpu(gpu, n, h, nH, x, pos, ndot, 1, **kw)
    assert rel_err(gm, ref)[0] <= 1e-4
    assert budget_err(bm, rb) <= 1e-6
    same_counts(bm, rb)


@pytest.mark.parametrize("periodic", [True, False])
@pytest.mark.parametrize("corr", [0, 1, 2, 3, 4])
def test_trace_mixed_matches_oracle(gpu, orc, periodic, corr):
    n = 24
    nH, x, pos, ndot, h = field_case(n, 200 + corr + 10 * periodic)
    kw = dict(periodic=periodic, n_min_ray=4.0, l_max=6, tau_max=25.0, n_th=4e-4, corr=corr)
    ref, rb = orc.trace(orc.make_params(n, h, **kw), nH, x, pos, ndot)
    got, b = run_gpu(gpu, n, h, nH, x, pos, ndot, 1, **kw)
    e_in, _ = rel_err(got, ref)
    assert e_in <= 1e-4, e_in
    E = b["emitted"]
    # A ray's transmitted share is a product of FP32 attenuation factors held
    # in FP64, and its children restart from e^{-tau} of the FP64 optical
    # depth: photons handed over at a split differ from those the parent
    # carried by that product's rounding drift (about 1e-7 relative per
    # split at most, random in sign), so E = A + X + T holds to ~1e-9 here
    assert abs(b["absorbed"] + b["escaped"] + b["truncated"] - E) <= 1e-8 * E
    assert budget_err(b, rb) <= 1e-6
    # every decision, the tau_max stop included, is FP64 and shared
    same_counts(b, rb)


def test_small_queues_chunk_and_recurse(gpu, orc):
    """A 4096-slot queue forces every level to be processed in many chunks,
    depth first; the result must not depend on the queue size."""
    n = 32
    nH, x, pos, ndot, h = field_case(n, 7, ionized=0.6, m=3, tau_cell=0.2)
    kw = dict(periodic=True, n_min_ray=4.0, l_max=7, tau_max=30.0, n_th=4e-4)
    ref, rb = orc.trace(orc.make_params(n, h, **kw), nH, x, pos, ndot)
    small, bs = run_gpu(gpu, n, h, nH, x, pos, ndot, 0, cap=4096, **kw)
    big, bb = run_gpu(gpu, n, h, nH, x, pos, ndot, 0, cap=1 << 20, **kw)
    assert max(rb["rays_per_level"]) > 4 * 4096
    for got, b in ((small, bs), (big, bb)):
        assert rel_err(got, ref)[0] <= 1e-10
        assert b["segments"] == rb["segments"] and b["rays"] == rb["rays"]
    np.testing.assert_allclose(small, big, rtol=1e-12, atol=1e-14 * big.max())


def test_edge_cases(gpu, orc):
    # no sources: Gamma = 0, empty budget
    n = 8
    nH, x = np.full((n, n, n), 1e-3), np.zeros((n, n, n))
    h = 1e20
    got, b = run_gpu(gpu, n, h, nH, x, np.zeros((0, 3)), np.zeros(0), 0)
    assert not got.any() and b["emitted"] == 0 and b["segments"] == 0
    # a one-cell grid, periodic and open
    for periodic in (True, False):
        kw = dict(periodic=periodic, n_min_ray=4.0, l_max=5, tau_max=30.0)
        one = (np.full((1, 1, 1), 1e-3), np.zeros((1, 1, 1)))
        ref, rb = orc.trace(orc.make_params(1, h, **kw), *one, [[0.3, 0.6, 0.9]], [1e49])
        got, b = run_gpu(gpu, 1, h, *one, [[0.3, 0.6, 0.9]], [1e49], 0, **kw)
        assert rel_err(got, ref)[0] <= 1e-12 and b["segments"] == rb["segments"]
    # structured ties: cell-centred and integer-coordinate sources, zero rate
    n = 16
    nH, x = np.full((n, n, n), 1e-3), np.zeros((n, n, n))
    x[4:12, 4:12, 4:12] = 1.0 - 1e-4
    pos = np.array([[8.5, 8.5, 8.5], [8.0, 8.0, 8.0], [0.0, 0.0, 0.0], [3.5, 12.0, 7.25]])
    ndot = np.array([1e50, 3e49, 2e49, 0.0])
    for periodic in (True, False):
        kw = dict(periodic=periodic, n_min_ray=4.0, l_max=6, tau_max=30.0, n_th=1e-5)
        ref, rb = orc.trace(orc.make_params(n, 2e20, **kw), nH, x, pos, ndot)
        got, b = run_gpu(gpu, n, 2e20, nH, x, pos, ndot, 0, **kw)
        assert rel_err(got, ref)[0] <= 1e-10
        assert b["segments"] == rb["segments"] and b["splits"] == rb["splits"]


def test_invalid_inputs_rejected(gpu):
    n = 8
    nH, x = np.full((n, n, n), 1e-3), np.zeros((n, n, n))
    d = gpu.make_desc(n, 1e20)
    bad = x.copy()
    bad[1, 2, 3] = 1.5
    with pytest.raises(gpu.NyxRTError) as e:
        gpu.init_grid(d, nH, bad, device="cuda:0", max_sources=4, ray_capacity=4096)
    assert e.value.status == 1
    ctx = gpu.init_grid(d, nH, x, device="cuda:0", max_sources=2, ray_capacity=4096)
    with pytest.raises(gpu.NyxRTError):
        ctx.add_sources([[8.0, 1.0, 1.0]], [1.0])  # outside [0, n)
    with pytest.raises(gpu.NyxRTError):
        ctx.add_sources([[1.0, 1.0, 1.0]], [-1.0])
    with pytest.raises(gpu.NyxRTError) as e:
        ctx.add_sources(np.ones((3, 3)), np.ones(3))  # table holds 2
    assert e.value.status == 4
    assert ctx.source_count() == 0
    with pytest.raises(gpu.NyxRTError):
        ctx.set_ionization(bad)
    # a rejected field leaves the context's field unchanged
    np.testing.assert_array_equal(ctx.get_ionization().cpu().numpy(), x)
    ctx.destroy()


@pytest.mark.slow
def test_full_lognormal_128_fp64_and_mixed(gpu, orc):
    """The 128^3 lognormal workload with all 64 sources at full size, in the
    launch configuration of the benchmark: FP64 against the oracle
    everywhere, mixed against the oracle, and source superposition."""
    w = W.config2()
    kw = dict(periodic=w.periodic, n_min_ray=w.n_min_ray, l_max=w.l_max, tau_max=w.tau_max,
              n_th=w.n_th)
    ref, rb = orc.trace(orc.make_params(w.n, w.h_cm, **kw), w.n_H, w.x, w.pos, w.ndot)
    got, b, _ = run_gpu_replayed(gpu, w, 0)
    assert rel_err(got, ref)[0] <= 1e-10
    assert b["segments"] == rb["segments"] and b["splits"] == rb["splits"]
    assert budget_err(b, rb) <= 1e-10
    gm, bm, _ = run_gpu_replayed(gpu, w, 1)
    assert rel_err(gm, ref)[0] <= 1e-4
    assert budget_err(bm, rb) <= 1e-6
    same_counts(bm, rb)
    # the host-driven chunked pass (small queues) executes the same segments
    gc, bc = run_gpu(gpu, w.n, w.h_cm, w.n_H, w.x, w.pos, w.ndot, 0, cap=1 << 21, **kw)
    assert bc["segments"] == rb["segments"] and rel_err(gc, ref)[0] <= 1e-10
    half = len(w.ndot) // 2
    g1, _ = run_gpu(gpu, w.n, w.h_cm, w.n_H, w.x, w.pos[:half], w.ndot[:half], 0, **kw)
    g2, _ = run_gpu(gpu, w.n, w.h_cm, w.n_H, w.x, w.pos[half:], w.ndot[half:], 0, **kw)
    np.testing.assert_allclose(g1 + g2, got, rtol=1e-12, atol=1e-13 * got.max())


@pytest.mark.parametrize("prec", [0, 1])
def test_rt_step_stromgren(gpu, orc, prec):
    """Config 1 (Stromgren Test A, Table testABCparams): all ten 2 Myr
    radiation steps on the GPU against the oracle's, in both precisions, and
    the ionized radius against the closed form (|r_n/r_a - 1| <= 0.10 after
    steps 1-2, <= 0.05 after steps 3-10).  After the first pass of a step
    the GPU replays the captured pass (absorber, trace, chemistry and the
    convergence check on the device)."""
    w = W.config1()
    kw = dict(periodic=False, n_min_ray=w.n_min_ray, l_max=w.l_max, tau_max=w.tau_max,
              n_th=w.n_th)
    alpha = w.extra["alpha_B"] * w.extra["clumping"]
    dt = w.extra["dt_s"]
    p = orc.make_params(w.n, w.h_cm, **kw)
    ctx = gpu.init_grid(gpu.make_desc(w.n, w.h_cm, precision=prec, **kw), w.n_H, w.x,
                        device="cuda:0", max_sources=1, ray_capacity=1 << 18)
    ctx.add_sources(w.pos, w.ndot)
    x_ref = w.x.copy()
    r_s = (3 * w.ndot[0] / (4 * math.pi * alpha * 1e-6)) ** (1 / 3) / w.h_cm
    t_rec = 1 / (alpha * 1e-3)
    replayed = 0
    for step in range(1, 11):
        x_ref, g_ref, b_ref, it_ref = orc.rt_step(p, w.n_H, x_ref, w.pos, w.ndot, dt, alpha)
        g, b, it = ctx.rt_step(dt, alpha)
        replayed += ctx.last_pass_was_graph()
        x_gpu = ctx.get_ionization().cpu().numpy()
        assert abs(it - it_ref) <= 1, (step, it, it_ref)
        if it == it_ref:
            assert np.abs(x_gpu - x_ref).max() <= (1e-6 if prec == 0 else 1e-4), step
        else:  # one pass apart at the threshold: keep the two in step
            ctx.set_ionization(x_ref)
            x_gpu = x_ref
        r_n = (3 * x_gpu.sum() / (4 * math.pi)) ** (1 / 3)
        r_a = r_s * (1 - math.exp(-step * dt / t_rec)) ** (1 / 3)
        assert r_n / r_a == pytest.approx(1.0, abs=0.10 if step <= 2 else 0.05), step
    assert replayed >= 5  # most steps take more than one pass
    ctx.destroy()


def test_rt_step_convergence_share(gpu, orc):
    """Radiation steps that stop once at most 0.1 % of the cells still move
    (conv_frac), on the GPU against the oracle with the same rule; invalid
    shares are rejected."""
    w = W.config1()
    kw = dict(periodic=False, n_min_ray=w.n_min_ray, l_max=w.l_max, tau_max=w.tau_max,
              n_th=w.n_th)
    alpha = w.extra["alpha_B"] * w.extra["clumping"]
    dt = w.extra["dt_s"]
    p = orc.make_params(w.n, w.h_cm, **kw)
    ctx = gpu.init_grid(gpu.make_desc(w.n, w.h_cm, **kw), w.n_H, w.x, device="cuda:0",
                        max_sources=1, ray_capacity=1 << 18)
    ctx.add_sources(w.pos, w.ndot)
    for bad in (-0.1, 1.5):
        with pytest.raises(gpu.NyxRTError):
            ctx.rt_step(dt, alpha, conv_frac=bad)
    x_ref = w.x.copy()
    for step in range(3):
        x_ref, _, _, it_ref = orc.rt_step(p, w.n_H, x_ref, w.pos, w.ndot, dt, alpha,
                                          conv_frac=1e-3)
        _, _, it = ctx.rt_step(dt, alpha, conv_frac=1e-3)
        assert abs(it - it_ref) <= 1, (step, it, it_ref)
        if it == it_ref:
            assert np.abs(ctx.get_ionization().cpu().numpy() - x_ref).max() <= 1e-6
        else:  # one pass apart near the threshold: keep the two in step
            ctx.set_ionization(x_ref)
    ctx.destroy()


def x_agrees(x, x_ref, moving, tol):
    """The ionized fractions of two radiation steps that stop once at most
    `moving` cells still move: those cells have not converged (the Gamma <-> x
    iteration there amplifies rounding differences between two
    implementations), so up to 2 * moving cells (either side's) may differ;
    every other cell agrees to tol."""
    d = np.sort(np.abs(x - x_ref).ravel())[::-1]
    return d[2 * moving] <= tol and d[0] <= 0.1, (d[0], d[2 * moving])


def test_rt_step_lognormal_64(gpu, orc):
    """Radiation steps at 64^3 (lognormal density, 4 bright sources that
    ionize the box, periodic): three 0.05 Myr steps that stop once at most
    1 % of the cells moved x by 1e-5 or more (the first takes ~26 passes, the
    next one each), GPU (FP64; mixed) against the oracle's: the same pass
    counts, and outside the cells still moving every x within 2 tol (both
    sides are within about tol of the same fixed point there) and within the
    precision's bar where that is larger."""
    n = 64
    g = np.random.default_rng(64)
    nH = W.lognormal_density(n, 1e-3, 1.0, g)
    x = np.zeros((n, n, n))
    pos = W.uniform_positions(4, n, g)
    ndot = W.lognormal_values(4, 3e49, 1.0, g)
    h = 0.3 / (W.SIGMA0 * 1e-3)
    kw = dict(periodic=True, n_min_ray=4.0, l_max=7, tau_max=30.0, n_th=1e-5)
    p = orc.make_params(n, h, **kw)
    dt, alpha, tol, frac, cap = 0.05 * W.MYR_S, W.ALPHA_B_1E4K, 1e-5, 1e-2, 60
    refs, x_ref = [], x.copy()
    for step in range(3):
        x_ref, _, _, it_ref = orc.rt_step(p, nH, x_ref, pos, ndot, dt, alpha, tol=tol,
                                          conv_frac=frac, max_iter=cap)
        assert it_ref < cap
        refs.append((x_ref, it_ref))
    for prec, bar in ((0, 2 * tol), (1, 1e-4)):
        ctx = gpu.init_grid(gpu.make_desc(n, h, precision=prec, **kw), nH, x, device="cuda:0",
                            max_sources=4, ray_capacity=1 << 21)
        ctx.add_sources(pos, ndot)
        for step, (xr, it_ref) in enumerate(refs):
            _, _, it = ctx.rt_step(dt, alpha, tol=tol, conv_frac=frac, max_iter=cap)
            assert abs(it - it_ref) <= 1, (prec, step, it, it_ref)
            if it == it_ref:
                ok, d = x_agrees(ctx.get_ionization().cpu().numpy(), xr, int(frac * n ** 3), bar)
                print(f"rt_step 64^3 prec {prec} step {step}: {it} passes, |dx| max {d[0]:.2e},"
                      f" beyond the moving cells {d[1]:.2e}", flush=True)
                assert ok, (prec, step, d)
            else:  # one pass apart at the threshold: keep the two in step
                ctx.set_ionization(xr)
        ctx.destroy()


@pytest.mark.slow
def test_rt_step_bubbles_256_subset(gpu, orc):
    """A radiation step on the 256^3 bubble field (16 of its 4096 sources,
    0.1 Myr, stopping once at most 0.1 % of the cells still move), in the
    benchmark's launch configuration, both precisions against the oracle's
    step: the same number of passes and the ionized fraction within 1e-6
    (FP64) / 1e-4 (mixed)."""
    import bench
    w = W.config3()
    s = W.subset(w, 16)
    kw = dict(periodic=w.periodic, n_min_ray=w.n_min_ray, l_max=w.l_max, tau_max=w.tau_max,
              n_th=w.n_th)
    dt, alpha = 0.1 * W.MYR_S, W.ALPHA_B_1E4K
    x_ref, _, _, it_ref = orc.rt_step(orc.make_params(w.n, w.h_cm, **kw), w.n_H, w.x, s.pos,
                                      s.ndot, dt, alpha, conv_frac=1e-3)
    print(f"bubbles-256 rt_step: oracle {it_ref} passes", flush=True)
    for prec, tol in ((0, 1e-6), (1, 1e-4)):
        ctx = gpu.init_grid(gpu.make_desc(w.n, w.h_cm, precision=prec, **kw), w.n_H, w.x,
                            device="cuda:0", max_sources=16, ray_capacity=BENCH_CAPACITY)
        refill, claim = bench.launch_params(w.name) or (0, 0)
        ctx.set_tuning(refill_min=refill, claim=claim)
        ctx.add_sources(s.pos, s.ndot)
        _, _, it = ctx.rt_step(dt, alpha, conv_frac=1e-3)
        ok, d = x_agrees(ctx.get_ionization().cpu().numpy(), x_ref, w.n ** 3 // 1000, tol)
        print(f"bubbles-256 rt_step prec {prec}: {it} passes, |dx| max {d[0]:.2e}, beyond the "
              f"moving cells {d[1]:.2e}", flush=True)
        assert it == it_ref and ok, (prec, it, it_ref, d)
        ctx.destroy()


@pytest.mark.slow
def test_bubbles_256_4096_sources(gpu, orc):
    """The 256^3 workload with 4096 sources in their own ionized bubbles, at
    full size in the benchmark's launch configuration (replayed device-driven
    pass): the mixed path against the FP64 path everywhere; both against the
    oracle on a seeded subset of 64 sources (Gamma is additive over sources
    for a fixed ionization field)."""
    w = W.config3()
    kw = dict(periodic=w.periodic, n_min_ray=w.n_min_ray, l_max=w.l_max, tau_max=w.tau_max,
              n_th=w.n_th)
    g64, b64, _ = run_gpu_replayed(gpu, w, 0)
    gmx, bmx, _ = run_gpu_replayed(gpu, w, 1)
    assert rel_err(gmx, g64)[0] <= 1e-4
    assert budget_err(bmx, b64) <= 1e-6
    same_counts(bmx, b64)
    E = b64["emitted"]
    assert abs(b64["absorbed"] + b64["escaped"] + b64["truncated"] - E) <= 1e-12 * E
    s = W.subset(w, 64)
    ref, rb = orc.trace(orc.make_params(w.n, w.h_cm, **kw), w.n_H, w.x, s.pos, s.ndot)
    gs, bs = run_gpu(gpu, w.n, w.h_cm, w.n_H, w.x, s.pos, s.ndot, 0, **kw)
    assert rel_err(gs, ref)[0] <= 1e-10
    assert bs["segments"] == rb["segments"] and bs["splits"] == rb["splits"]
    gm, bm = run_gpu(gpu, w.n, w.h_cm, w.n_H, w.x, s.pos, s.ndot, 1, **kw)
    assert rel_err(gm, ref)[0] <= 1e-4
    assert budget_err(bm, rb) <= 1e-6
    same_counts(bm, rb)


@pytest.mark.parametrize("prec", [0, 1])
def test_tuning_changes_only_speed(gpu, orc, prec):
    """Launch parameters (run size, refill threshold, resident blocks, graph
    mode) and the autotuner's choice execute the same segments, rays and
    splits and give the same Gamma (to the summation order of the deposits:
    1e-12 FP64, FP32 partial sums 2e-5 mixed)."""
    n = 32
    nH, x, pos, ndot, h = field_case(n, 77, ionized=0.3, m=5, tau_cell=0.3)
    kw = dict(periodic=True, n_min_ray=4.0, l_max=7, tau_max=30.0, n_th=4e-4)
    ref, rb = orc.trace(orc.make_params(n, h, **kw), nH, x, pos, ndot)
    ctx = gpu.init_grid(gpu.make_desc(n, h, precision=prec, **kw), nH, x, device="cuda:0",
                        max_sources=8, ray_capacity=1 << 21)
    ctx.add_sources(pos, ndot)
    g0, b0 = ctx.trace_step()
    base = g0.cpu().numpy()
    assert rel_err(base, ref)[0] <= (1e-10 if prec == 0 else 1e-4)
    rtol = 1e-12 if prec == 0 else 2e-5
    for refill, claim, bpc, graph in [(1, 64, 1, 1), (64, 65536, 0, 1), (8, 256, 2, 2),
                                      (32, 1024, 0, 0), (0, 0, 0, 0)]:
        ctx.set_tuning(refill, claim, bpc, graph)
        for _ in range(2):  # the second pass may replay a captured graph
            g, b = ctx.trace_step(g0)
            for k in ("segments", "rays", "splits", "rays_per_level"):
                assert b[k] == b0[k], (refill, claim, bpc, graph, k)
            np.testing.assert_allclose(g.cpu().numpy(), base, rtol=rtol, atol=1e-14 * base.max())
    best = ctx.autotune(passes=1, gamma=g0)
    assert set(best) == {"refill_min", "claim", "blocks_per_cu", "graph"}
    g, b = ctx.trace_step(g0)
    assert b["segments"] == b0["segments"]
    np.testing.assert_allclose(g.cpu().numpy(), base, rtol=rtol, atol=1e-14 * base.max())
    ctx.destroy()


@pytest.mark.slow
def test_clustered_512_merged(gpu, orc):
    """The merged 512^3 clustered catalogue (32768 sources) at full size in
    the benchmark's launch configuration: the GPU's merged catalogue equals
    the oracle's; the mixed path against the FP64 path over the whole
    catalogue; both against the oracle on a seeded subset of 64 merged
    sources."""
    w = W.config4()
    kw = dict(periodic=w.periodic, n_min_ray=w.n_min_ray, l_max=w.l_max, tau_max=w.tau_max,
              n_th=w.n_th)
    g64, b64, (p, f, _) = run_gpu_replayed(gpu, w, 0, merge=True)
    gmx, bmx, _ = run_gpu_replayed(gpu, w, 1, merge=True)
    mc, mf, _ = orc.merge_sources(orc.make_merge_params(), w.n, w.periodic, w.x, w.pos, w.ndot)
    np.testing.assert_array_equal(np.floor(p).astype(np.int32), mc)
    np.testing.assert_allclose(f, mf, rtol=1e-13, atol=0)
    assert rel_err(gmx, g64)[0] <= 1e-4
    assert budget_err(bmx, b64) <= 1e-6
    same_counts(bmx, b64)
    E = b64["emitted"]
    assert abs(b64["absorbed"] + b64["escaped"] + b64["truncated"] - E) <= 1e-12 * E
    idx = np.sort(np.random.default_rng(512).choice(len(mf), size=64, replace=False))
    sp, sf = mc[idx] + 0.5, mf[idx]
    ref, rb = orc.trace(orc.make_params(w.n, w.h_cm, **kw), w.n_H, w.x, sp, sf)
    gs, bs = run_gpu(gpu, w.n, w.h_cm, w.n_H, w.x, sp, sf, 0, **kw)
    assert rel_err(gs, ref)[0] <= 1e-10
    assert bs["segments"] == rb["segments"] and bs["splits"] == rb["splits"]
    gm, bm = run_gpu(gpu, w.n, w.h_cm, w.n_H, w.x, sp, sf, 1, **kw)
    assert rel_err(gm, ref)[0] <= 1e-4
    assert budget_err(bm, rb) <= 1e-6
    same_counts(bm, rb)


def test_graph_replays_match_eager_passes(gpu, orc):
    """Once a pass shows every level fits its queue, later passes replay a
    captured device-driven pass (hipGraph).  Every replay, with eager work
    and synchronisation between them, must equal the eager chunked pass and
    the oracle; changing the sources or the output buffer re-captures; a
    queue too small for a level falls back to the chunked pass."""
    import torch
    n = 32
    nH, x, pos, ndot, h = field_case(n, 51, ionized=0.4, m=6, tau_cell=0.3)
    kw = dict(periodic=True, n_min_ray=4.0, l_max=7, tau_max=30.0, n_th=4e-4)
    ref, rb = orc.trace(orc.make_params(n, h, **kw), nH, x, pos, ndot)
    # The mixed path sums its deposits in FP32 LDS slots whose order of
    # arrival varies from pass to pass, so replays agree to FP32 rounding of
    # those partial sums (all terms positive: relative error <= k * 2^-24 for
    # k deposits per slot between flushes); the FP64 path to 1e-12.
    for prec, tol, rep_tol in ((0, 1e-10, 1e-12), (1, 1e-4, 2e-5)):
        ctx = gpu.init_grid(gpu.make_desc(n, h, precision=prec, **kw), nH, x, device="cuda:0",
                            max_sources=16, ray_capacity=1 << 21)
        ctx.add_sources(pos, ndot)
        g_eager, b_eager = ctx.trace_step()
        assert not ctx.last_pass_was_graph()
        eager = g_eager.cpu().numpy()
        assert rel_err(eager, ref)[0] <= tol
        for rep in range(4):
            junk = torch.randn(1 << 20, device="cuda:0").sum()  # eager work in between
            torch.cuda.synchronize()
            g, b = ctx.trace_step(g_eager)
            assert ctx.last_pass_was_graph(), rep
            got = g.cpu().numpy()
            np.testing.assert_allclose(got, eager, rtol=rep_tol, atol=1e-14 * eager.max())
            for k in ("segments", "rays", "splits", "rays_per_level"):
                assert b[k] == b_eager[k], (rep, k)
            assert abs(b["absorbed"] - b_eager["absorbed"]) <= 1e-12 * b["emitted"]
            del junk
        # a new output buffer and a changed source list are captured again
        g2, b2 = ctx.trace_step()
        assert ctx.last_pass_was_graph()
        np.testing.assert_allclose(g2.cpu().numpy(), eager, rtol=rep_tol,
                                   atol=1e-14 * eager.max())
        ctx.add_sources(pos[:2], ndot[:2])
        ref2, rb2 = orc.trace(orc.make_params(n, h, **kw), nH, x, np.vstack([pos, pos[:2]]),
                              np.concatenate([ndot, ndot[:2]]))
        g3, b3 = ctx.trace_step()
        assert rel_err(g3.cpu().numpy(), ref2)[0] <= tol
        ctx.destroy()
    # forced graph with a queue too small: overflow, then the chunked pass
    ctx = gpu.init_grid(gpu.make_desc(n, h, **kw), nH, x, device="cuda:0", max_sources=16,
                        ray_capacity=4096)
    ctx.add_sources(pos, ndot)
    ctx.set_tuning(graph=2)
    g, b = ctx.trace_step()
    assert not ctx.last_pass_was_graph()
    assert rel_err(g.cpu().numpy(), ref)[0] <= 1e-10 and b["segments"] == rb["segments"]
    ctx.destroy()


def rel_err_dev(got, ref, floor=1e-6):
    """rel_err for two torch tensors on the GPU (the 1024^3 fields)."""
    mask = ref > floor * ref.max()
    e_in = float((got[mask] / ref[mask] - 1).abs().max()) if bool(mask.any()) else 0.0
    e_out = (float((got[~mask] - ref[~mask]).abs().max()) / float(ref.max())
             if bool((~mask).any()) else 0.0)
    return e_in, e_out


@pytest.mark.slow
def test_late_reion_1024_merged(gpu, orc):
    """The 1024^3 late-reionization workload (262 144 clustered sources in
    5000 overlapping bubbles, merged) at full size in the benchmark's launch
    configuration (2^27-slot level queues, host-driven chunks): the GPU's
    merged catalogue equals the oracle's; the mixed path against the FP64
    path over the whole merged catalogue, with equal counts; both paths
    against the oracle on a seeded subset of 2 merged sources (each casts
    about 3e8 segments through the 70 % ionized volume, and the oracle runs
    one thread at this grid size)."""
    import torch
    import bench
    w = W.config5()
    kw = dict(periodic=w.periodic, n_min_ray=w.n_min_ray, l_max=w.l_max, tau_max=w.tau_max,
              n_th=w.n_th)
    mc, mf, _ = orc.merge_sources(orc.make_merge_params(), w.n, w.periodic, w.x, w.pos, w.ndot)
    print(f"late-reion-1024: oracle merged {len(w.ndot)} -> {len(mf)} sources", flush=True)
    idx = np.sort(np.random.default_rng(1024).choice(len(mf), size=2, replace=False))
    sp, sf = mc[idx] + 0.5, mf[idx]
    ref, rb = orc.trace(orc.make_params(w.n, w.h_cm, **kw), w.n_H, w.x, sp, sf)
    print(f"late-reion-1024: oracle subset {rb['segments']} segments", flush=True)
    refill, claim = bench.launch_params(w.name)
    full = {}
    for prec in (0, 1):
        ctx = gpu.init_grid(gpu.make_desc(w.n, w.h_cm, precision=prec, **kw), w.n_H, w.x,
                            device="cuda:0", max_sources=len(w.ndot),
                            ray_capacity=bench.DEFAULT_CAPACITY[w.name])
        ctx.set_tuning(refill_min=refill, claim=claim)
        ctx.add_sources(w.pos, w.ndot)
        ctx.merge_sources(gpu.make_merge_params())
        p, f, _ = ctx.get_sources()
        np.testing.assert_array_equal(np.floor(p).astype(np.int32), mc)
        np.testing.assert_allclose(f, mf, rtol=1e-13, atol=0)
        g, b = ctx.trace_step()
        E = b["emitted"]
        assert abs(b["absorbed"] + b["escaped"] + b["truncated"] - E) <= \
            (1e-10 if prec == 0 else 1e-8) * E
        full[prec] = (g, b)
        print(f"late-reion-1024 prec {prec}: full pass {b['segments']} segments", flush=True)
        ctx.clear_sources()
        ctx.add_sources(sp, sf)
        gs, bs = ctx.trace_step()
        got = gs.cpu().numpy()
        del gs
        ctx.destroy()
        del ctx
        torch.cuda.empty_cache()  # each context holds ~160 GB of queues
        e_in, e_out = rel_err(got, ref)
        print(f"late-reion-1024 prec {prec}: subset vs oracle {e_in:.2e} / {e_out:.2e}",
              flush=True)
        tol = 1e-10 if prec == 0 else 1e-4
        assert e_in <= tol and e_out <= tol, (prec, e_in, e_out)
        # the oracle adds this subset's ~5.6e8 per-segment absorptions in one
        # thread, one after another: its rounding bound is ~n u = 6e-8 of the
        # total (measured against the GPU's blocked sums: 1.1e-10)
        assert budget_err(bs, rb) <= (1e-8 if prec == 0 else 1e-6)
        same_counts(bs, rb)
        del got
    (g64, b64), (gmx, bmx) = full[0], full[1]
    same_counts(bmx, b64)
    assert budget_err(bmx, b64) <= 1e-6
    e_in, e_out = rel_err_dev(gmx, g64)
    print(f"late-reion-1024: mixed vs FP64 {e_in:.2e} / {e_out:.2e}", flush=True)
    assert e_in <= 1e-4 and e_out <= 1e-4, (e_in, e_out)
    del full, g64, gmx
    torch.cuda.empty_cache()
