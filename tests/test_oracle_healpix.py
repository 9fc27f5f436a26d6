"""Pins for the oracle's HEALPix pixel centres.

The paper splits rays along the nested HEALPix hierarchy (Sec. "Adaptive ray
tracing", Fig. raysplit).  What fixes the pixelisation is Gorski et al.
(2005): 12 N_side^2 equal-area pixels on 4 N_side - 1 iso-latitude rings,
ring heights 1 - i^2/(3 N_side^2) in the caps and 4/3 - 2i/(3 N_side) in the
belt, pixels equally spaced in phi on each ring, and the nested numbering in
which pixel p at level l owns pixels 4p .. 4p+3 at level l+1.  The inverse
map below (ang2pix, nested) is written independently of the oracle from the
same publication and used to check the hierarchy.
"""
import math

import numpy as np
import pytest


def _interleave(ix, iy, level):
    p = 0
    for b in range(level):
        p |= ((ix >> b) & 1) << (2 * b)
        p |= ((iy >> b) & 1) << (2 * b + 1)
    return p


def ang2pix_nest(level, v):
    """Nested pixel containing direction v (Gorski et al. 2005)."""
    ns = 1 << level
    z = v[2] / math.sqrt(v[0] ** 2 + v[1] ** 2 + v[2] ** 2)
    phi = math.atan2(v[1], v[0])
    tt = (phi / (0.5 * math.pi)) % 4.0
    za = abs(z)
    if za <= 2.0 / 3.0:
        t1 = ns * (0.5 + tt)
        t2 = ns * z * 0.75
        jp = int(t1 - t2)
        jm = int(t1 + t2)
        ifp, ifm = jp // ns, jm // ns
        if ifp == ifm:
            face = (ifp % 4) + 4
        elif ifp < ifm:
            face = ifp % 4
        else:
            face = (ifm % 4) + 8
        ix = jm & (ns - 1)
        iy = ns - (jp & (ns - 1)) - 1
    else:
        ntt = min(3, int(tt))
        tp = tt - ntt
        tmp = ns * math.sqrt(3.0 * (1.0 - za))
        jp = min(int(tp * tmp), ns - 1)
        jm = min(int((1.0 - tp) * tmp), ns - 1)
        if z >= 0:
            face, ix, iy = ntt, ns - jm - 1, ns - jp - 1
        else:
            face, ix, iy = ntt + 8, jp, jm
    return face * ns * ns + _interleave(ix, iy, level)


def test_level0_exact(orc):
    d = orc.healpix_dirs(0)
    s5 = math.sqrt(5.0) / 3.0  # sin(theta) at z = 2/3
    for p in range(4):  # north: z = 2/3, phi = pi/4 + p pi/2
        phi = math.pi / 4 + p * math.pi / 2
        np.testing.assert_allclose(d[p], [s5 * math.cos(phi), s5 * math.sin(phi), 2 / 3],
                                   atol=1e-15)
        np.testing.assert_allclose(d[p + 8], [s5 * math.cos(phi), s5 * math.sin(phi), -2 / 3],
                                   atol=1e-15)
        phi = p * math.pi / 2  # equator
        np.testing.assert_allclose(d[p + 4], [math.cos(phi), math.sin(phi), 0.0], atol=1e-15)
    # structured values are exact
    assert d[4][1] == 0.0 and d[5][0] == 0.0 and d[4][2] == 0.0
    assert abs(d[0][0]) == abs(d[0][1])


@pytest.mark.parametrize("level", [0, 1, 2, 3, 4, 5])
def test_counts_norms_and_balance(orc, level):
    d = orc.healpix_dirs(level)
    assert d.shape == (12 * 4 ** level, 3)
    np.testing.assert_allclose(np.linalg.norm(d, axis=1), 1.0, atol=2e-16 * 4)
    assert len(np.unique(d, axis=0)) == d.shape[0]
    np.testing.assert_allclose(d.sum(0), 0.0, atol=1e-12)


@pytest.mark.parametrize("level", [1, 2, 3, 4])
def test_ring_structure(orc, level):
    """4 N_side - 1 rings; ring heights and pixel counts of Gorski et al. 2005;
    pixels equally spaced in phi on each ring with the published offsets."""
    ns = 1 << level
    d = orc.healpix_dirs(level)
    z = d[:, 2]
    rings = {}
    for i in range(1, 4 * ns):
        if i < ns:
            zi, cnt, off = 1 - i * i / (3 * ns * ns), 4 * i, 0.5
        elif i > 3 * ns:
            k = 4 * ns - i
            zi, cnt, off = -(1 - k * k / (3 * ns * ns)), 4 * k, 0.5
        else:
            zi, cnt = 4 / 3 - 2 * i / (3 * ns), 4 * ns
            off = 0.5 if (i - ns) % 2 == 0 else 1.0
        rings[i] = (zi, cnt, off)
    assigned = np.zeros(len(z), bool)
    for i, (zi, cnt, off) in rings.items():
        sel = np.abs(z - zi) < 1e-13
        assert sel.sum() == cnt, (i, sel.sum(), cnt)
        assigned |= sel
        phi = np.sort(np.mod(np.arctan2(d[sel, 1], d[sel, 0]), 2 * np.pi))
        expect = np.sort(np.mod((np.arange(1, cnt + 1) - off) * 2 * np.pi / cnt, 2 * np.pi))
        np.testing.assert_allclose(phi, expect, atol=1e-12)
    assert assigned.all()


@pytest.mark.parametrize("level", [0, 1, 2, 3, 4])
def test_nested_hierarchy(orc, level):
    """Each pixel centre maps to itself, and each of the 4 children of pixel
    p (4p .. 4p+3 at level+1) maps back to p, under ang2pix_nest."""
    d = orc.healpix_dirs(level)
    dc = orc.healpix_dirs(level + 1)
    for p in range(d.shape[0]):
        assert ang2pix_nest(level, d[p]) == p
        for k in range(4):
            assert ang2pix_nest(level, dc[4 * p + k]) == p
            assert ang2pix_nest(level + 1, dc[4 * p + k]) == 4 * p + k


@pytest.mark.parametrize("level", [0, 1, 2, 3, 4])
def test_exact_mirror_symmetry(orc, level):
    """Mirror images (x,y,z)->(x,y,-z), (-x,y,z), (y,x,z) of pixel centres
    are pixel centres, bit for bit."""
    d = orc.healpix_dirs(level)
    S = {tuple(v) for v in (d + 0.0)}  # + 0.0 folds -0.0 into 0.0
    for v in d + 0.0:
        for w in ((v[0], v[1], -v[2]), (-v[0], v[1], v[2]), (v[1], v[0], v[2])):
            w = tuple(np.array(w) + 0.0)
            assert w in S
