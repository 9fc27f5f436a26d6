"""The entry point that allocates nothing (nrt_trace_step_noalloc) against
nrt_trace_step on the same inputs, through the C ABI: two calls in a row,
the second with a smaller grid and fewer sources, in both precisions.  Both
run the same kernels (the no-allocation form keeps its state in the
library's static device scratch), so the bar is the oracle bar between
them: FP64 within 1e-10, mixed within 1e-4 where Gamma > 1e-6 max, budget
terms within 1e-10 / 1e-6 of the emitted rate, counts equal."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def case(n, seed, m):
    g = np.random.default_rng(seed)
    nH = W.lognormal_density(n, 1e-3, 1.0, g)
    x = np.where(g.random((n, n, n)) < 0.3, 1.0 - 1e-4, 0.0)
    pos = W.uniform_positions(m, n, g)
    ndot = W.lognormal_values(m, 1e50, 1.0, g)
    return nH, x, pos, ndot, 0.4 / (W.SIGMA0 * 1e-3)


def rel(got, ref):
    mask = ref > 1e-6 * ref.max()
    return float(np.abs(got[mask] / ref[mask] - 1).max())


@pytest.mark.parametrize("prec", [0, 1])
def test_noalloc_matches_trace_step(gpu, prec):
    import torch
    for n, m, seed in ((40, 5, 1), (24, 2, 2)):  # the second call is smaller
        nH, x, pos, ndot, h = case(n, seed, m)
        kw = dict(periodic=True, n_min_ray=4.0, l_max=6, tau_max=30.0, n_th=4e-4,
                  precision=prec)
        desc = gpu.make_desc(n, h, **kw)
        ctx = gpu.init_grid(desc, nH, x, device="cuda:0", max_sources=m, ray_capacity=1 << 20)
        ctx.add_sources(pos, ndot)
        g_ref, b_ref = ctx.trace_step()
        ref = g_ref.cpu().numpy()
        ctx.destroy()
        # queues as wide as the widest level (the device-driven pass has no
        # chunked fallback)
        cap = max(4096, 1 << int(np.ceil(np.log2(max(b_ref["rays_per_level"])))))
        assert cap <= 1 << 18
        dev = torch.device("cuda:0")
        nh_t = torch.from_numpy(nH).to(dev)
        x_t = torch.from_numpy(x).to(dev)
        gamma = torch.full((n, n, n), float("nan"), dtype=torch.float64, device=dev)
        b = gpu.trace_step_noalloc(desc, nh_t, x_t, pos, ndot, gamma, cap)
        got = gamma.cpu().numpy()
        assert np.isfinite(got).all()
        tol = 1e-10 if prec == 0 else 1e-4
        assert rel(got, ref) <= tol, (n, rel(got, ref))
        for k in ("segments", "rays", "splits", "rays_per_level"):
            assert b[k] == b_ref[k], (n, k)
        E = b_ref["emitted"]
        assert abs(b["emitted"] - E) <= 1e-15 * E
        for k in ("absorbed", "escaped", "truncated"):
            assert abs(b[k] - b_ref[k]) <= (1e-10 if prec == 0 else 1e-6) * E, (n, k)


def test_noalloc_rejects_what_does_not_fit(gpu):
    import torch
    n = 8
    dev = torch.device("cuda:0")
    f = torch.zeros((n, n, n), dtype=torch.float64, device=dev)
    g = torch.empty_like(f)
    desc = gpu.make_desc(n, 1e20, l_max=10)
    with pytest.raises(gpu.NyxRTError) as e:  # 10 levels of 2^20 slots: 240 MiB
        gpu.trace_step_noalloc(desc, f + 1e-3, f, [[1.0, 1.0, 1.0]], [1e49], g, 1 << 20)
    assert e.value.status == 3
    with pytest.raises(gpu.NyxRTError) as e:
        gpu.trace_step_noalloc(gpu.make_desc(n, 1e20, spectrum=1, spec_param=5e4), f + 1e-3, f,
                               [[1.0, 1.0, 1.0]], [1e49], g, 4096)
    assert e.value.status == 1
