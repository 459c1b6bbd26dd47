"""The serving replay's request arena (bench.py): first-fit ranges of one
buffer.  Over random allocation and release sequences, live ranges never
overlap, stay inside the buffer and are 256-byte aligned; free ranges stay
sorted, disjoint and merged with their neighbours; and live plus free bytes
always equal the buffer.  No device is needed: the ranges are bookkeeping."""
import random

import bench


def arena(nbytes):
    a = bench.RequestArena.__new__(bench.RequestArena)   # no device buffer
    a.free = [(0, nbytes)]
    return a


def check(a, live, cap):
    free = a.free
    assert free == sorted(free)
    for (o1, s1), (o2, s2) in zip(free, free[1:]):
        assert o1 + s1 < o2, "free ranges must be disjoint and merged"
    spans = sorted([(o, a._round(n)) for o, n in live.values()] + free)
    assert spans[0][0] == 0 and spans[-1][0] + spans[-1][1] == cap
    for (o1, s1), (o2, s2) in zip(spans, spans[1:]):
        assert o1 + s1 == o2, "live and free ranges tile the buffer"
    for o, n in live.values():
        assert o % 256 == 0 and o + n <= cap


def test_random_sequences_keep_the_invariants():
    cap = 1 << 22
    for seed in range(5):
        rng = random.Random(seed)
        a = arena(cap)
        live = {}
        for t in range(4000):
            if live and rng.random() < 0.45:
                k = rng.choice(sorted(live))
                o, n = live.pop(k)
                a.release(o, n)
            else:
                n = rng.randint(1, cap // 20)
                o = a.alloc(n)
                if o is not None:
                    live[t] = (o, n)
            check(a, live, cap)
        for k in sorted(live):
            a.release(*live.pop(k))
        assert a.free == [(0, cap)]


def test_first_fit_and_refusal():
    a = arena(4096)
    x = a.alloc(1000)       # rounds to 1024
    y = a.alloc(1024)
    z = a.alloc(2048)
    assert (x, y, z) == (0, 1024, 2048)
    assert a.alloc(1) is None   # full
    a.release(y, 1024)
    assert a.alloc(2000) is None   # the hole is 1024 bytes
    assert a.alloc(700) == 1024    # first fit takes 768 bytes of the hole
    a.release(x, 1000)
    a.release(z, 2048)             # merges with the hole's 256-byte rest
    assert a.free == [(0, 1024), (1792, 2304)]
