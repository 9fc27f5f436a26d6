"""Brute-force geometry used to pin the oracle's cell traversal.

A ray o + t d crosses cell (i,j,k) on the interval where it is inside all
three slabs [i, i+1) x [j, j+1) x [k, k+1) (the slab method for ray/box
intersection).  Enumerating every cell in a bounding range and sorting the
non-empty intervals gives the exact cell sequence and segment lengths that a
voxel traversal (Amanatides & Woo, cited in Sec. "User-defined filter and
transform functions") must reproduce.
"""
import math

import numpy as np


def slab_interval(o, d, lo, hi):
    """[t0, t1] of the ray inside the axis-aligned box [lo, hi]; None if empty."""
    t0, t1 = -math.inf, math.inf
    for a in range(3):
        if d[a] == 0.0:
            if not (lo[a] <= o[a] < hi[a]):
                return None
            continue
        ta = (lo[a] - o[a]) / d[a]
        tb = (hi[a] - o[a]) / d[a]
        if ta > tb:
            ta, tb = tb, ta
        t0, t1 = max(t0, ta), min(t1, tb)
    if t1 < t0:
        return None
    return t0, t1


def box_exit(o, d, n):
    """Distance from o (inside [0,n)^3) to where the ray leaves the box."""
    iv = slab_interval(o, d, (0.0, 0.0, 0.0), (float(n),) * 3)
    return iv[1]


def cells_along(o, d, t_start, t_stop, min_len=1e-9):
    """Unwrapped cells crossed with positive length for t in [t_start, t_stop]
    (cells entered at t < t_stop), as a list of (ijk, t0, t1) sorted by t0."""
    o = np.asarray(o, float)
    d = np.asarray(d, float)
    p0 = o + t_start * d
    p1 = o + t_stop * d
    lo = np.floor(np.minimum(p0, p1)).astype(int) - 1
    hi = np.floor(np.maximum(p0, p1)).astype(int) + 1
    out = []
    for i in range(lo[0], hi[0] + 1):
        for j in range(lo[1], hi[1] + 1):
            for k in range(lo[2], hi[2] + 1):
                iv = slab_interval(o, d, (i, j, k), (i + 1, j + 1, k + 1))
                if iv is None:
                    continue
                t0, t1 = max(iv[0], t_start), iv[1]
                if t1 - t0 <= min_len or t0 >= t_stop:
                    continue
                out.append(((i, j, k), t0, t1))
    out.sort(key=lambda e: e[1])
    return out
