"""Host logic of the serving loop (no GPU): the photon-range allocator."""
import random

from paper_1303_5057_amd.serve import ALIGN, RangeAllocator


def test_allocator_first_fit_alignment_and_merge():
    a = RangeAllocator(1024)
    x = a.alloc(100)
    y = a.alloc(64)
    z = a.alloc(1)
    assert (x, y, z) == (0, 128, 192)
    assert a.used() == 256
    a.release(y, 64)
    assert a.alloc(60) == 128          # first fit reuses the hole
    a.release(x, 100)
    a.release(128, 60)
    a.release(z, 1)
    assert a.free == [[0, 1024]] and a.used() == 0
    assert a.alloc(2000) is None


def test_allocator_random_never_overlaps():
    rng = random.Random(5)
    a = RangeAllocator(64 * 500)
    live = {}
    for step in range(4000):
        if live and rng.random() < 0.45:
            k = rng.choice(list(live))
            a.release(k, live.pop(k))
        else:
            n = rng.randint(1, 64 * 40)
            s = a.alloc(n)
            if s is not None:
                assert s % ALIGN == 0
                live[s] = n
        spans = sorted((s, s + (n + ALIGN - 1) // ALIGN * ALIGN) for s, n in live.items())
        for (s0, e0), (s1, e1) in zip(spans, spans[1:]):
            assert e0 <= s1
        assert all(e <= a.capacity for _, e in spans)
        assert a.used() == sum(e - s for s, e in spans)
