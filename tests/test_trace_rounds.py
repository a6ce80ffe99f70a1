"""The schedule of a TRACE shared by many workgroups in place (no second
register): outputs in rounds [0, 2^(p+1)), then [2^k, 2^(k+1)) for
k = p+1 .. b-3, output j written on entry j.  Checked here for every register
width up to 2^11 and every bit pair: no output of a round lands on an entry
that another output of the same round reads, and running the rounds in order,
each round's outputs in any order, leaves the trace in entries 0 .. 2^(b-2)-1."""

import numpy as np


def insert_zero(x, bit):
    return (x & ((1 << bit) - 1)) | ((x >> bit) << (bit + 1))


def rounds(b, p):
    nb = b - 2
    k0 = min(p + 1, nb)
    return [(0, k0)] + [(1 << k, k) for k in range(k0, nb)]


def test_rounds_cover_the_outputs_once():
    for b in range(3, 12):
        for p in range(b - 1):
            r = rounds(b, p)
            cover = np.concatenate([np.arange(lo, lo + (1 << k)) for lo, k in r])
            assert np.array_equal(np.sort(cover), np.arange(1 << (b - 2))), (b, p)


def test_no_output_lands_on_another_outputs_input_within_a_round():
    for b in range(3, 12):
        for p in range(b):
            for q in range(p + 1, b):
                step = (1 << p) + (1 << q)
                j = np.arange(1 << (b - 2))
                i0 = insert_zero(insert_zero(j, p), q)
                reader = np.full(1 << b, -1)
                reader[i0] = j
                reader[i0 + step] = j
                for lo, k in rounds(b, p):
                    out = np.arange(lo, lo + (1 << k))
                    r = reader[out]
                    assert np.all((r < 0) | (r == out) | (r < lo)), (b, p, q, lo)


def test_rounds_in_order_give_the_trace():
    rng = np.random.default_rng(3)
    for b in range(3, 12):
        for p in range(b):
            for q in range(p + 1, b):
                step = (1 << p) + (1 << q)
                j = np.arange(1 << (b - 2))
                i0 = insert_zero(insert_zero(j, p), q)
                reg = rng.standard_normal(1 << b)
                want = reg[i0] + reg[i0 + step]
                for lo, k in rounds(b, p):
                    for o in rng.permutation(np.arange(lo, lo + (1 << k))):
                        reg[o] = reg[i0[o]] + reg[i0[o] + step]
                assert np.array_equal(reg[: 1 << (b - 2)], want), (b, p, q)
