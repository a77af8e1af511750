"""Oracle values of a weighted-sum chain on a window of a large grid."""
import numpy as np

import oracle


def window_oracle(ch, data, centre, half):
    """Oracle values of the chain's final datasets on a window around `centre`:
    the chain runs on a crop of the padded arrays with every loop's range
    shrunk by the largest stencil radius per loop, so the centre region
    [centre - (half - 2L), centre + (half - 2L)) is exact."""
    nd, n, h, L = ch.ndim, ch.n, ch.halo, len(ch.loops)
    lo = [max(c - half, -h) for c in centre]
    hi = [min(c + half, n + h) for c in centre]
    sl = tuple(slice(l + h, u + h) for l, u in zip(reversed(lo), reversed(hi)))
    crop = [np.ascontiguousarray(a[sl]) for a in data]
    # a grid whose "halo" offset maps logical lo to index 0
    arrs = [a.copy() for a in crop]

    class W(oracle.Grid):
        def view(self, a):
            v = super().view(a)
            v.origin = -(lo[0] * 1 + (lo[1] * a.shape[-1] if nd > 1 else 0) +
                         (lo[2] * a.shape[-1] * a.shape[-2] if nd > 2 else 0))
            return v

    g = W(nd, n, 0)
    for l, lp in enumerate(ch.loops):
        m = 2 * (l + 1)
        rlo = [0 if a == -h else max(0, a + m) for a in lo]
        rhi = [n if b == n + h else min(n, b - m) for b in hi]
        if any(b <= a for a, b in zip(rlo, rhi)):
            continue
        oracle.wsum(g, rlo, rhi, arrs[lp.out], [arrs[c.dat] for c in lp.inputs],
                    [c.stencil for c in lp.inputs], lp.weights)
    m = 2 * L
    good_lo = [max(0, a + m) if a > -h else 0 for a in lo]
    good_hi = [min(n, b - m) if b < n + h else n for b in hi]
    return arrs, lo, good_lo, good_hi


def euler_window(q, n, h, zlo, zhi, dt, gamma=1.4, halo=2, margin=8):
    """Oracle RK3 step of a 3D Euler state restricted to the planes
    [zlo, zhi): the step runs on a z-crop of the padded arrays with `margin`
    extra planes each side (three stages of a radius-2 stencil need 6).
    Returns (Q after the step, R of the last stage), each a list of arrays
    (z in [zlo, zhi), all y and x including halos)."""
    import ctypes
    from oracle import OV, Grid, lib
    from oracle.euler import RK3
    clo, chi = max(zlo - margin, -halo), min(zhi + margin, n + halo)
    crop = [np.ascontiguousarray(a[clo + halo:chi + halo]) for a in q]
    D = 3

    class ZGrid(Grid):
        def view(self, a):
            v = super().view(a)
            v.origin = -clo * a.shape[1] * a.shape[2] + halo * a.shape[2] + halo
            return v

    g = ZGrid(D, n, halo)
    L = lib()
    qs = [a.copy() for a in crop]
    q0 = [a.copy() for a in crop]
    vel = [np.zeros_like(crop[0]) for _ in range(D)]
    p = np.zeros_like(crop[0])
    r = [np.zeros_like(crop[0]) for _ in range(D + 2)]

    def views(arrs):
        return (OV * len(arrs))(*[g.view(a) for a in arrs])

    plo, phi = g.box([-halo, -halo, clo], [n + halo, n + halo, chi])
    ilo, ihi = g.box([0, 0, max(clo + 2, 0)], [n, n, min(chi - 2, n)])
    s = 1.0 / (12.0 * h)
    for a, b in RK3:
        L.orc_euler_prim(D, plo, phi, views(qs), views(vel), g.view(p), ctypes.c_double(gamma - 1.0))
        for c in range(D + 2):
            L.orc_euler_rhs(D, ilo, ihi, c, g.view(r[c]), g.view(qs[c]), views(vel), g.view(p), ctypes.c_double(s))
        for c in range(D + 2):
            L.orc_rk_stage(ilo, ihi, g.view(q0[c]), g.view(qs[c]), g.view(r[c]), ctypes.c_double(a),
                           ctypes.c_double(b), ctypes.c_double(dt))
    sl = slice(zlo - clo, zhi - clo)
    return [a[sl] for a in qs], [a[sl] for a in r]


def jacobi_window(u0, iters, points, weights, copy, y0, x0, s):
    """Oracle values of the Jacobi iteration on the s x s block of interior
    cells [y0, y0 + s) x [x0, x0 + s) of a large field u0 ((n+2)^2, the
    Dirichlet layer included).  A cell after T iterations depends only on
    cells within distance T, so the oracle runs on the crop that extends the
    block by T cells per side (clipped at the real layer), whose outer ring
    stays fixed.  Where the ring is a cut through the interior its stale
    values reach at most T cells inwards, never the block."""
    from oracle.jacobi import jacobi
    n = u0.shape[0] - 2
    ya, yb = max(y0 - iters, 0), min(y0 + s + iters, n)
    xa, xb = max(x0 - iters, 0), min(x0 + s + iters, n)
    # interior coordinate c is array index c + 1; the crop keeps one ring
    crop = np.ascontiguousarray(u0[ya:yb + 2, xa:xb + 2])
    out = jacobi(crop, iters, points, weights, copy)
    return out[y0 - ya + 1:y0 - ya + 1 + s, x0 - xa + 1:x0 - xa + 1 + s]
