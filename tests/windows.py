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
