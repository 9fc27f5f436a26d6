"""Seeded synthetic inputs for the ray-tracing sweep.

This module holds only input generation (density and ionization fields,
source catalogues and the named workload configurations).  It contains none
of the method's arithmetic, and both the GPU path's tests/benchmark and the
oracle take their inputs from here.

The paper's workloads are Nyx cosmological fields (a 40 h^-1 cMpc periodic box,
ray tracing on 256^3 .. 1024^3 coarse grids, sources from a halo finder) and
the Stromgren Test A of Table testABCparams.  None of that data exists here,
so lognormal density fields, bubble ionization fields and clustered sources
stand in, with the paper's grid sizes, periodicity and physical
normalisation.

Seeds: numpy ``default_rng(12466 + 100 * cfg + stream)``; stream 0 = density,
1 = source positions, 2 = luminosities, 3 = bubbles.
"""
import math
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field
from typing import Optional

import numpy as np
import scipy.fft as sfft

SEED_BASE = 12466
KPC_CM = 3.0856775814913673e21
MPC_CM = 3.0856775814913673e24
MYR_S = 3.15576e13
SIGMA0 = 6.30e-18            # H photo-ionisation cross-section at 13.6 eV, cm^2
ALPHA_B_1E4K = 2.59e-13      # Table testABCparams caption, cm^3 s^-1

# cosmology of the paper's large runs (Sec. "Simulation parameters"), at z = 7
_H = 0.67742
_OMEGA_B = 0.0488911
_CHI_H = 0.76                 # hydrogen mass fraction (the paper does not state it)
_M_P = 1.67262192e-24
_RHO_CRIT0 = 1.87847e-29 * _H * _H   # g cm^-3
Z_RT = 7.0
NH_COSMO = _CHI_H * _OMEGA_B * _RHO_CRIT0 * (1.0 + Z_RT) ** 3 / _M_P   # ~9.8e-5 cm^-3
L_BOX_COSMO_CM = 40.0 / _H / (1.0 + Z_RT) * MPC_CM                     # ~7.38 Mpc physical


def rng(cfg: int, stream: int) -> np.random.Generator:
    return np.random.default_rng(SEED_BASE + 100 * cfg + stream)


_SLAB = 16  # planes of the first axis per generation task


def _threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def _over_slabs(n: int, fn) -> list:
    """fn(lo, hi) for the slabs [lo, hi) of the first axis, on a thread pool
    (numpy releases the GIL in bulk array work); results in slab order."""
    spans = [(lo, min(n, lo + _SLAB)) for lo in range(0, n, _SLAB)]
    with ThreadPoolExecutor(_threads()) as ex:
        return list(ex.map(lambda sp: fn(*sp), spans))


def gaussian_field(n: int, gen: np.random.Generator, slope: float = -2.0,
                   log=None) -> np.ndarray:
    """Periodic Gaussian random field with power spectrum P(k) ~ k^slope,
    zero mean, unit variance, shape (n,n,n) indexed [k,j,i].

    White noise comes from one child generator per slab of _SLAB planes
    (seeded from `gen`), so the field does not depend on the thread count."""
    log = log or (lambda *a: None)
    seeds = np.random.SeedSequence(int(gen.integers(0, 2 ** 63))).spawn((n + _SLAB - 1) // _SLAB)
    white = np.empty((n, n, n))

    def fill(lo, hi):
        np.random.default_rng(seeds[lo // _SLAB]).standard_normal(out=white[lo:hi])
    _over_slabs(n, fill)
    log("gaussian field: white noise done")
    fk = sfft.rfftn(white, workers=_threads())
    del white
    log("gaussian field: forward FFT done")
    kx = np.fft.fftfreq(n) * n
    kz = np.fft.rfftfreq(n) * n

    # sqrt(P) = k^(slope/2), applied one plane of the first axis at a time
    def shape(lo, hi):
        for a in range(lo, hi):
            k2 = kx[a] ** 2 + kx[:, None] ** 2 + kz[None, :] ** 2
            with np.errstate(divide="ignore"):
                fk[a] *= np.where(k2 > 0, k2 ** (slope / 4.0), 0.0)
    _over_slabs(n, shape)
    log("gaussian field: spectrum applied")
    g = sfft.irfftn(fk, s=(n, n, n), axes=(0, 1, 2), workers=_threads())
    del fk
    log("gaussian field: inverse FFT done")
    # zero mean, unit variance: per-slab sums combined in slab order
    mean = sum(_over_slabs(n, lambda lo, hi: float(g[lo:hi].sum()))) / g.size

    def centre(lo, hi):
        g[lo:hi] -= mean
        return float(np.square(g[lo:hi]).sum())
    std = math.sqrt(sum(_over_slabs(n, centre)) / g.size)

    def scale(lo, hi):
        g[lo:hi] /= std
    _over_slabs(n, scale)
    return g


def lognormal_density(n: int, mean: float, sigma_ln: float, gen, log=None) -> np.ndarray:
    """n_H = mean * exp(sigma g - sigma^2 / 2): lognormal with the given mean."""
    g = gaussian_field(n, gen, log=log)

    def ln(lo, hi):
        v = g[lo:hi]
        v *= sigma_ln
        v -= 0.5 * sigma_ln ** 2
        np.exp(v, out=v)
        v *= mean
    _over_slabs(n, ln)
    return g


def lognormal_values(m: int, mean: float, sigma_ln: float, gen) -> np.ndarray:
    return mean * np.exp(sigma_ln * gen.standard_normal(m) - 0.5 * sigma_ln ** 2)


def uniform_positions(m: int, n: int, gen) -> np.ndarray:
    """Continuous positions uniform in [0, n)^3 (cell units)."""
    p = gen.random((m, 3)) * n
    return np.minimum(p, np.nextafter(float(n), 0.0))


def clustered_cells(n: int, n_clusters: int, per_cluster: int, sigma_cells: float, gen):
    """Cluster centres uniform in the box; members = centre + N(0, sigma^2) per
    axis, wrapped and snapped to the cell, returned as cell centres.
    Returns (positions (m,3), centres (n_clusters,3))."""
    centres = gen.random((n_clusters, 3)) * n
    off = gen.standard_normal((n_clusters, per_cluster, 3)) * sigma_cells
    p = (centres[:, None, :] + off).reshape(-1, 3)
    cells = np.floor(p).astype(np.int64) % n
    return cells.astype(np.float64) + 0.5, centres


def paint_bubbles(n: int, centres: np.ndarray, radii: np.ndarray, x_in: float = 1.0 - 1e-4,
                  periodic: bool = True, out: Optional[np.ndarray] = None) -> np.ndarray:
    """Ionized fraction: x_in in every cell whose centre lies within a
    bubble (min-image distance <= r), 0 elsewhere.  Shape (n,n,n) [k,j,i].
    Threads paint disjoint slabs of the first axis, so the result does not
    depend on the thread count (every painted cell gets the same value)."""
    x = np.zeros((n, n, n)) if out is None else out
    boxes = []
    for c, r in zip(np.asarray(centres, float), np.asarray(radii, float)):
        lo = np.floor(c - r - 1).astype(int)
        hi = np.ceil(c + r + 1).astype(int)
        ii = [np.arange(lo[a], hi[a] + 1) for a in range(3)]
        if not periodic:
            ii = [v[(v >= 0) & (v < n)] for v in ii]
        if not all(v.size for v in ii):
            continue
        d = [(v + 0.5 - c[a]) ** 2 for a, v in enumerate(ii)]
        inside = (d[2][:, None, None] + d[1][None, :, None] + d[0][None, None, :]) <= r * r
        boxes.append(([v % n for v in (ii[2], ii[1], ii[0])], inside))

    def paint(k0, k1):
        for (kk, jj, iq), inside in boxes:
            sel = (kk >= k0) & (kk < k1)
            if not sel.any():
                continue
            sub = x[np.ix_(kk[sel], jj, iq)]
            sub[inside[sel]] = x_in
            x[np.ix_(kk[sel], jj, iq)] = sub
    _over_slabs(n, paint)
    return x


def _radius_scale(n, centres, u, share, gen, samples=400000, log=None):
    """Smallest rho with bubbles of radii rho*u covering `share` of the
    volume, from a Monte-Carlo sample of cell centres: a sample point lies
    in some bubble iff min_b d_b / u_b <= rho (periodic min-image distance
    d_b), so the covered share at rho is the share of points whose minimum
    is at most rho, and rho is that minimum's `share`-quantile.  Bubbles are
    taken in blocks on a thread pool; a minimum does not depend on order."""
    pts = np.floor(gen.random((samples, 3)) * n) + 0.5
    centres = np.asarray(centres, float)
    u = np.asarray(u, float)
    block = 32

    def part(b0):
        q = np.full(samples, np.inf)
        for c, ub in zip(centres[b0:b0 + block], u[b0:b0 + block]):
            d = np.abs(pts - c)
            d = np.minimum(d, n - d)
            np.minimum(q, np.sqrt((d * d).sum(1)) / ub, out=q)
        return q
    with ThreadPoolExecutor(_threads()) as ex:
        parts = list(ex.map(part, range(0, centres.shape[0], block)))
    q = np.minimum.reduce(parts)
    if log:
        log(f"radius scale: {centres.shape[0]} bubbles")
    return float(np.quantile(q, share, method="inverted_cdf"))


@dataclass
class Workload:
    name: str
    n: int
    h_cm: float
    periodic: bool
    n_H: np.ndarray
    x: np.ndarray
    pos: np.ndarray
    ndot: np.ndarray
    n_min_ray: float
    l_max: int
    tau_max: float
    n_th: float
    merge: bool = False
    extra: dict = field(default_factory=dict)

    def params(self, **over):
        d = dict(n=self.n, h_cm=self.h_cm, periodic=self.periodic, sigma0=SIGMA0,
                 n_min_ray=self.n_min_ray, l_max=self.l_max, tau_max=self.tau_max,
                 n_th=self.n_th)
        d.update(over)
        return d


def config1() -> Workload:
    """Stromgren Test A (Table testABCparams): n_H = 1e-3, Ndot = 5e48, C = 1,
    L_box = 6.6 kpc, T = 1e4 K; 32^3 cells, one source at the centre of cell
    (16,16,16), open boundaries."""
    n = 32
    return Workload("stromgren-testA-32", n, 6.6 * KPC_CM / n, False,
                    np.full((n, n, n), 1e-3), np.zeros((n, n, n)),
                    np.array([[16.5, 16.5, 16.5]]), np.array([5e48]),
                    n_min_ray=4.0, l_max=7, tau_max=30.0, n_th=1e-5,
                    extra=dict(alpha_B=ALPHA_B_1E4K, clumping=1.0, dt_s=2.0 * MYR_S, steps=10))


def config2(n: int = 128, m: int = 64) -> Workload:
    """128^3 lognormal density (ln-sigma 1, P(k) ~ k^-2), mean n_H = 1e-3,
    neutral, 64 uniform sources with lognormal rates (mean 1e50/s, ln-sigma 1),
    periodic; the cell width makes the mean neutral cell optical depth 0.5."""
    h = 0.5 / (SIGMA0 * 1e-3) * (128 / n)
    nH = lognormal_density(n, 1e-3, 1.0, rng(2, 0))
    pos = uniform_positions(m, n, rng(2, 1))
    ndot = lognormal_values(m, 1e50, 1.0, rng(2, 2))
    return Workload(f"lognormal-{n}-{m}src", n, h, True, nH, np.zeros((n, n, n)), pos, ndot,
                    n_min_ray=4.0, l_max=9, tau_max=30.0, n_th=1e-5)


def config3(n: int = 256, m: int = 4096) -> Workload:
    """256^3 lognormal density (ln-sigma 1.5) at the cosmological mean n_H of
    z = 7, 4096 uniform sources, rates lognormal (ln-sigma 2), one ionized
    bubble per source of radius clip(6 (Ndot/mean)^(1/3), 2, 32) cells."""
    h = L_BOX_COSMO_CM / n
    nH = lognormal_density(n, NH_COSMO, 1.5, rng(3, 0))
    pos = uniform_positions(m, n, rng(3, 1))
    ndot = lognormal_values(m, 1e50, 2.0, rng(3, 2))
    radii = np.clip(6.0 * (ndot / 1e50) ** (1.0 / 3.0), 2.0, 32.0) * (n / 256)
    x = paint_bubbles(n, pos, radii)
    return Workload(f"lognormal-{n}-{m}src-bubbles", n, h, True, nH, x, pos, ndot,
                    n_min_ray=4.0, l_max=10, tau_max=30.0, n_th=1e-2 * NH_COSMO)


def config4(n: int = 512, n_clusters: int = 512, per_cluster: int = 64,
            n_bubbles: int = 200) -> Workload:
    """512^3 lognormal (ln-sigma 1.5), 512 clusters x 64 cell-snapped sources
    (sigma = 2 cells), 200 bubbles r ~ U[4,20] centred on random cluster
    centres; merging on."""
    h = L_BOX_COSMO_CM / n
    nH = lognormal_density(n, NH_COSMO, 1.5, rng(4, 0))
    pos, centres = clustered_cells(n, n_clusters, per_cluster, 2.0, rng(4, 1))
    ndot = lognormal_values(pos.shape[0], 1e50, 2.0, rng(4, 2))
    g = rng(4, 3)
    pick = g.choice(n_clusters, size=min(n_bubbles, n_clusters), replace=False)
    radii = g.uniform(4.0, 20.0, size=pick.size)
    x = paint_bubbles(n, centres[pick], radii)
    return Workload(f"clustered-{n}-{pos.shape[0]}src", n, h, True, nH, x, pos, ndot,
                    n_min_ray=4.0, l_max=11, tau_max=30.0, n_th=1e-2 * NH_COSMO, merge=True)


def config5(n: int = 1024, n_clusters: int = 4096, per_cluster: int = 64,
            n_bubbles: int = 5000, target: float = 0.70, log=None) -> Workload:
    """1024^3 lognormal (ln-sigma 1.5), 4096 clusters x 64 sources, 5000
    bubbles (4096 on cluster centres + 904 uniform) with r = rho U[0.5,1.5],
    rho chosen so that the bubbles cover the target ionized volume share;
    merging on.  `log` (optional) receives a line per generation phase."""
    log = log or (lambda *a: None)
    h = L_BOX_COSMO_CM / n
    nH = lognormal_density(n, NH_COSMO, 1.5, rng(5, 0), log=log)
    log("config5: density done")
    pos, centres = clustered_cells(n, n_clusters, per_cluster, 2.0, rng(5, 1))
    ndot = lognormal_values(pos.shape[0], 1e50, 2.0, rng(5, 2))
    g = rng(5, 3)
    extra_c = g.random((n_bubbles - n_clusters, 3)) * n
    bc = np.concatenate([centres, extra_c])
    u = g.uniform(0.5, 1.5, size=bc.shape[0])
    rho = _radius_scale(n, bc, u, target, np.random.default_rng(SEED_BASE + 599), log=log)
    log(f"config5: radius scale {rho:.3f}")
    x = np.zeros((n, n, n))
    for k in range(0, bc.shape[0], 1000):
        paint_bubbles(n, bc[k:k + 1000], rho * u[k:k + 1000], out=x)
        log(f"config5: painted {min(k + 1000, bc.shape[0])} bubbles")
    return Workload(f"late-reion-{n}-{pos.shape[0]}src", n, h, True, nH, x, pos, ndot,
                    n_min_ray=4.0, l_max=10, tau_max=30.0, n_th=1e-2 * NH_COSMO, merge=True,
                    extra=dict(rho=rho))


CONFIGS = {1: config1, 2: config2, 3: config3, 4: config4, 5: config5}


def subset(w: Workload, k: int, seed: int = 7) -> Workload:
    """The same workload restricted to a seeded random subset of k sources
    (the trace is additive over sources for a fixed ionization field)."""
    g = np.random.default_rng(SEED_BASE + 900 + seed)
    idx = np.sort(g.choice(w.pos.shape[0], size=min(k, w.pos.shape[0]), replace=False))
    return Workload(w.name + f"-sub{len(idx)}", w.n, w.h_cm, w.periodic, w.n_H, w.x,
                    w.pos[idx].copy(), w.ndot[idx].copy(), w.n_min_ray, w.l_max, w.tau_max,
                    w.n_th, w.merge, dict(w.extra, subset=idx))
