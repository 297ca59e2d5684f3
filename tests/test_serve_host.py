"""CPU checks of the serving loop's host logic: the arena allocator and the
seeded request stream (no GPU)."""
import random

import numpy as np

from paper_1209_5198_amd import serve, synth


def test_arena_first_fit_never_overlaps_and_coalesces():
    a = serve.Arena(1 << 20, device=None)
    live = []
    rng = random.Random(1)
    for _ in range(5000):
        if live and rng.random() < 0.5:
            o, w = live.pop(rng.randrange(len(live)))
            a.release(o, w)
        else:
            w = rng.randint(1, 50000)
            o = a.alloc(w)
            if o is None:
                assert a.cap - a.used < serve.Arena.size(w) or len(a.free) > 1
                continue
            assert o % serve.GRANULE == 0 and o + serve.Arena.size(w) <= a.cap
            for o2, w2 in live:
                assert o + serve.Arena.size(w) <= o2 or o2 + serve.Arena.size(w2) <= o
            live.append((o, w))
        assert a.used == sum(serve.Arena.size(w) for _, w in live)
    for o, w in live:
        a.release(o, w)
    assert a.free == [(0, a.cap)] and a.used == 0


def test_arena_full_cap_waits():
    a = serve.Arena(4096, device=None)
    o1 = a.alloc(4000)
    assert o1 == 0 and a.alloc(200) is None
    a.release(o1, 4000)
    assert a.alloc(4096) == 0


def test_serving_specs_shapes_and_kinds():
    sp = synth.serving_specs(5, 3000)
    assert sp == synth.serving_specs(5, 3000)  # deterministic
    kinds = [s["kind"] for s in sp]
    for k in synth.SERVE_KINDS:
        assert 0.28 < kinds.count(k) / len(sp) < 0.39
    sq = [s for s in sp if s["n"] == s["m"]]
    rect = [s for s in sp if s["n"] != s["m"]]
    assert 0.44 < len(sq) / len(sp) < 0.56
    assert all(128 <= s["n"] <= 16384 for s in sq)
    for s in rect:
        lo_, hi_ = sorted((s["n"], s["m"]))
        assert hi_ // 4 == lo_ and 512 <= hi_ <= 16384
    # log-uniform: the median square side is near sqrt(128 * 16384) = 1448
    med = np.median([s["n"] for s in sq])
    assert 1000 < med < 2100


def test_poisson_arrivals_rate():
    a = synth.poisson_arrivals(9, 20000, 500.0)
    assert np.all(np.diff(a) > 0)
    assert abs(a[-1] / 20000 - 1 / 500.0) < 0.05 / 500.0 * 3
    gaps = np.diff(np.concatenate([[0.0], a]))
    assert abs(np.std(gaps) * 500.0 - 1.0) < 0.05  # exponential: sd = mean
