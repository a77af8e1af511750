"""Pins of the oracle's weighted-sum chain executor.

The chain is linear in the stacked datasets, so on tiny grids it equals the
product of one sparse matrix per loop (assembled here with scipy from flat
indices, a formulation independent of the oracle's strided C loops).  A wrong
stencil direction, a transposed offset or a dropped term changes the product.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from synthgen import make_chain, chain_data, star


def flat_index(shape, coord_zyx):
    idx = 0
    for s, c in zip(shape, coord_zyx):
        idx = idx * s + c
    return idx


def loop_matrix(ch, lp):
    shape = ch.shape_alloc
    size = int(np.prod(shape))
    nd, h, n = ch.ndim, ch.halo, ch.n
    rows, cols, vals = [], [], []
    written = set()
    for pt in np.ndindex(*([n] * nd)):           # pt in (z, y, x) order, interior
        coord = tuple(c + h for c in pt)
        r = lp.out * size + flat_index(shape, coord)
        written.add(r)
        q = 0
        for ci in lp.inputs:
            for off in ci.stencil:                 # off is (x, y[, z])
                off_zyx = tuple(reversed(off))
                src = tuple(c + o for c, o in zip(coord, off_zyx))
                rows.append(r)
                cols.append(ci.dat * size + flat_index(shape, src))
                vals.append(lp.weights[q])
                q += 1
    total = ch.ndat * size
    keep = [i for i in range(total) if i not in written]
    rows += keep
    cols += keep
    vals += [1.0] * len(keep)
    return sp.csr_matrix((vals, (rows, cols)), shape=(total, total))


@pytest.mark.parametrize("ndim,n,ndat,nloops", [(2, 7, 4, 6), (3, 5, 5, 5), (2, 9, 12, 12)])
def test_chain_equals_sparse_product(ndim, n, ndat, nloops):
    ch = make_chain(ndim, n, ndat, nloops, seed=100 + ndim)
    data = chain_data(ch)
    got = oracle.run_chain(ch, data)
    s = np.concatenate([a.ravel() for a in data])
    for lp in ch.loops:
        s = loop_matrix(ch, lp) @ s
    want = s.reshape(ch.ndat, -1)
    for d in range(ch.ndat):
        err = np.abs(got[d].ravel() - want[d]).max()
        assert err <= 1e-14 * max(1.0, np.abs(want[d]).max())


def test_constant_field_closed_form():
    """All datasets constant c: every output equals c * (sum of the loop's weights)
    as long as its inputs are still constant."""
    ch = make_chain(2, 6, 3, 1, seed=5)
    data = [np.full(ch.shape_alloc, 0.75) for _ in range(ch.ndat)]
    got = oracle.run_chain(ch, data)
    lp = ch.loops[0]
    want = 0.75 * np.sum(lp.weights)
    g = oracle.Grid(2, ch.n, ch.halo)
    assert np.allclose(oracle.interior(g, got[lp.out]), want, rtol=1e-15, atol=0)
    # untouched datasets and halos keep their values
    for d in range(ch.ndat):
        if d != lp.out:
            assert np.array_equal(got[d], data[d])
    h = ch.halo
    assert np.all(got[lp.out][:h, :] == 0.75)


def test_single_point_stencil_shift():
    """One input, one stencil point (+1 in x) with weight 1: a pure shift."""
    from synthgen import SyntheticChain, ChainLoop, ChainInput
    ch = SyntheticChain(2, 5, 2, 2, [ChainLoop(1, [ChainInput(0, [(1, 0)])], [1.0])], 0)
    a = np.arange(81, dtype=np.float64).reshape(9, 9)
    got = oracle.run_chain(ch, [a, np.zeros((9, 9))])
    assert np.array_equal(got[1][2:7, 2:7], a[2:7, 3:8])
    ch.loops[0].inputs[0].stencil = [(0, -2)]
    got = oracle.run_chain(ch, [a, np.zeros((9, 9))])
    assert np.array_equal(got[1][2:7, 2:7], a[0:5, 2:7])


def test_exact_sum_and_dot():
    import math
    vals = np.array([1e16, 1.0, -1e16, 1e-3])
    assert oracle.exact_sum(vals) == math.fsum(vals.tolist()) == 1.001
    rng = np.random.default_rng(0)
    a = rng.standard_normal(1000)
    b = rng.standard_normal(1000)
    from fractions import Fraction
    exact = sum(Fraction(x) * Fraction(y) for x, y in zip(a.tolist(), b.tolist()))
    g = oracle.Grid(1, 1000, 0)
    c = np.empty(2000)
    L = oracle.lib()
    import ctypes
    lo, hi = g.box([0], [1000])
    L.orc_dot_terms(lo, hi, g.view(a), g.view(b), c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    assert oracle.exact_dot_terms(c) == float(exact)


def test_window_oracle_equals_full_oracle():
    """The windowed evaluation used to sample full-size GPU results is exact."""
    from windows import window_oracle
    ch = make_chain(2, 150, 6, 20, seed=8)
    data = chain_data(ch)
    ref = oracle.run_chain(ch, data)
    for c in [(0, 0), (149, 149), (75, 2), (60, 100)]:
        arrs, lo, glo, ghi = window_oracle(ch, data, c, 60)
        for d in range(ch.ndat):
            got = ref[d][glo[1] + 2:ghi[1] + 2, glo[0] + 2:ghi[0] + 2]
            want = arrs[d][glo[1] - lo[1]:ghi[1] - lo[1], glo[0] - lo[0]:ghi[0] - lo[0]]
            assert got.size > 0 and np.array_equal(got, want)
