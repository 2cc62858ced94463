"""Host logic of the serving loop's workspace arena (first fit over a sorted
free list of 256-byte granules, merged on release): random allocate/release
sequences keep the free list and the live ranges an exact partition of the
arena, with no two free ranges adjacent."""
import random

import torch

from paper_2608_24348_amd.serve import _Arena


def test_arena_partition_under_random_traffic():
    a = _Arena(torch, 1 << 20, "cpu")
    rng = random.Random(1)
    live = []
    for _ in range(20000):
        if live and rng.random() < 0.5:
            a.release(*live.pop(rng.randrange(len(live))))
        else:
            got = a.alloc(rng.randrange(1, 50000))
            if got:
                live.append(got)
        free = a.free
        assert all(free[i][0] + free[i][1] < free[i + 1][0] for i in range(len(free) - 1))
        pos = 0
        for o, n in sorted(live + [tuple(x) for x in free]):
            assert o == pos and o % 256 == 0 and n % 256 == 0
            pos = o + n
        assert pos == a.size
    for o, n in live:
        a.release(o, n)
    assert a.empty()


def test_arena_views_are_aligned_and_refuse_oversize():
    a = _Arena(torch, 10000, "cpu")
    assert a.alloc(a.size + 1) is None
    o, n = a.alloc(300)
    assert n == 512 and a.view(o, n).data_ptr() % 256 == 0 and a.view(o, n).numel() == n
