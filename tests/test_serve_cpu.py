"""Host-side parts of the serving loop: the arena allocator, the footprint
used for admission, and the Poisson arrival schedule."""
from __future__ import annotations

import numpy as np

from paper_2103_00154_amd import dsg, inputs, serve


def test_arena_first_fit_and_coalescing():
    a = serve.Arena(10 * 256 + 100)
    assert a.size == 10 * 256
    x = a.alloc(1)
    y = a.alloc(300)          # two granules
    z = a.alloc(256)
    assert (x, y, z) == (0, 256, 768)
    assert a.used == 4 * 256
    a.free(y, 300)
    assert a.alloc(600) == 1024  # the hole of two granules is too small
    assert a.alloc(512) == 256   # but fits two
    a.free(256, 512)
    a.free(x, 1)
    a.free(z, 256)
    a.free(1024, 600)
    assert a.used == 0 and a._free == [(0, 10 * 256)]
    assert a.alloc(10 * 256) == 0 and a.alloc(1) is None
    assert a.peak == 10 * 256


def test_arena_random_alloc_free_keeps_blocks_disjoint():
    rng = np.random.default_rng(0)
    a = serve.Arena(1 << 20)
    live = {}
    for step in range(3000):
        if live and rng.random() < 0.45:
            off = list(live)[rng.integers(len(live))]
            a.free(off, live.pop(off))
        else:
            nb = int(rng.integers(1, 40_000))
            off = a.alloc(nb)
            if off is not None:
                live[off] = nb
        spans = sorted((o, o + (nb + 255) // 256 * 256) for o, nb in live.items())
        assert all(s1[1] <= s2[0] for s1, s2 in zip(spans, spans[1:]))
        assert a.used == sum(e - o for o, e in spans)
    for off, nb in list(live.items()):
        a.free(off, nb)
    assert a._free == [(0, 1 << 20)]


def test_footprint_covers_the_batch_workspace_share():
    # a request's footprint must cover what it adds to a batch: CSR, output
    # slots and workspace (per-vertex arrays, one table row, tile entries)
    for n, m in ((100, 300), (20_000, 400_000), (1_000_000, 30_000_000)):
        one = dsg.batch_workspace_bytes(1, 2 * m, n)
        assert serve.footprint(n, m) >= 4 * (n + 1 + 2 * m) + 4 * n + one - 256


def test_poisson_arrivals_rate():
    t = serve.poisson_arrivals(20_000, 1000.0, seed=3)
    assert np.all(np.diff(t) > 0)
    assert abs(len(t) / t[-1] - 1000.0) < 30


def test_serving_specs_follow_the_recipe():
    specs = inputs.serving_specs(2000, seed=0)
    n = np.array([s.n for s in specs])
    assert n.min() >= 100 and n.max() <= 2_000_000
    assert 15_000 < np.median(n) < 26_000
    assert all(s.kind == inputs.KIND_CHUNG_LU for s in specs)
    d = np.array([s.avg_deg for s in specs])
    assert d.min() >= 8 and d.max() <= 64
