"""Pins of the shared seeded input generator."""
import numpy as np

from synthgen import SplitMix64, splitmix_block, uniform_block, make_chain, star, batch_sizes, serving_requests


def test_splitmix64_reference_outputs():
    # first outputs of SplitMix64 from state 0, as published with the generator
    r = SplitMix64(0)
    assert [r.next() for _ in range(3)] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    assert [int(v) for v in splitmix_block(0, 0, 3)] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4,
                                                         0x06C45D188009454F]


def test_counter_form_matches_sequential():
    r = SplitMix64(12345)
    seq = [r.next() for _ in range(50)]
    assert [int(v) for v in splitmix_block(12345, 0, 50)] == seq
    assert [int(v) for v in splitmix_block(12345, 20, 5)] == seq[20:25]


def test_uniform_ranges():
    u = uniform_block(7, 0, 100000, -1.0, 1.0)
    assert u.min() >= -1.0 and u.max() < 1.0 and abs(u.mean()) < 0.01


def test_star_stencils():
    assert len(star(2, 1)) == 5 and len(star(2, 2)) == 9
    assert len(star(3, 1)) == 7 and len(star(3, 2)) == 13
    assert star(2, 2)[3] == (-2, 0)


def test_chain_structure():
    ch = make_chain(2, 64, 12, 40, seed=1)
    assert len(ch.loops) == 40
    for lp in ch.loops:
        ins = [c.dat for c in lp.inputs]
        assert 2 <= len(ins) <= 4 and len(set(ins)) == len(ins) and lp.out not in ins
        assert len(lp.weights) == sum(len(c.stencil) for c in lp.inputs)
        assert all(-0.25 <= w < 0.25 for w in lp.weights)


def test_batch_and_serving_draws():
    b = batch_sizes(512, 3)
    assert len(b) == 512 and all(64 <= n <= 1024 for n, _ in b)
    reqs = serving_requests(200.0, 5.0, 4)
    assert 800 < len(reqs) < 1200
    assert all(a.arrival < b.arrival for a, b in zip(reqs, reqs[1:]))
