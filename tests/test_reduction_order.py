"""The kinetic-energy reduction order, emulated on the host: the drift
kernel's last block (256 slots) over at most 64 block partials takes the
same sums, in the same order, as the 1024-slot tree of the separate reduce
kernel, so the two launch forms give the same E_k bit for bit."""
import numpy as np
import pytest


def tree(vals, slots):
    red = np.zeros(slots)
    red[:len(vals)] = vals
    w = slots // 2
    while w > 0:
        red[:w] = red[:w] + red[w:2 * w]
        w //= 2
    return red[0]


def reduce_kernel(partials):
    # thread t sums partials t, t + 1024, ... in order, then the 1024-slot tree
    s = np.zeros(1024)
    for b, x in enumerate(partials):
        s[b % 1024] = s[b % 1024] + x
    return tree(s, 1024)


@pytest.mark.parametrize("nblk", [1, 2, 3, 17, 40, 63, 64])
def test_last_block_sum_equals_the_reduce_kernel(nblk):
    rng = np.random.default_rng(nblk)
    for _ in range(50):
        # partials of very different sizes, so that any other order rounds differently
        p = rng.random(nblk) * 10.0 ** rng.integers(-12, 3, nblk)
        assert tree(p, 256).tobytes() == reduce_kernel(p).tobytes()


def test_a_different_order_would_show():
    # the emulation can tell orders apart: summing left to right differs
    rng = np.random.default_rng(0)
    differ = 0
    for _ in range(200):
        p = rng.random(64) * 10.0 ** rng.integers(-12, 3, 64)
        seq = 0.0
        for x in p:
            seq += x
        differ += seq != reduce_kernel(p)
    assert differ > 0
