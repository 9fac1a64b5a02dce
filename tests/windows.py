"""Windowed oracle for sampled parity checks on large grids."""
import numpy as np

from oracle.tfan_oracle import Oracle


def window_oracle(p, ic, cx, cy, half, steps, radius=12):
    """The oracle on a periodic window around (cx, cy): after `steps` steps the
    central (2 half)^2 block is exact, since one step depends on at most `radius`
    sites in each direction."""
    nx, ny = p["nx"], p["ny"]
    R = half + radius * steps
    xs = np.arange(cx - R, cx + R) % nx
    ys = np.arange(cy - R, cy + R) % ny
    w = dict(p, nx=2 * R, ny=2 * R)
    o = Oracle(w)
    o.init_fields(*(ic[k][np.ix_(ys, xs)] for k in ("phi", "qxx", "qxy")))
    o.step(steps)
    f = o.get_fields()
    sl = slice(R - half, R + half)
    return {k: (v[..., sl, sl]) for k, v in f.items()}, xs[sl], ys[sl]
