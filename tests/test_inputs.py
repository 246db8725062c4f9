"""The seeded input generators: reproducible, distinct, first-drawn order."""
import numpy as np

from paper_2209_00117_amd import inputs


def test_place_seeds_is_sequential_rejection():
    """The vectorised placement equals the plain sequential loop: draw
    (x, y) pairs from the stream and keep a pair only if its pixel is free."""
    for (W, H, S, seed) in [(7, 5, 35, 3), (64, 48, 300, 1), (512, 512, 256, 1)]:
        got = inputs.place_seeds(W, H, S, seed)
        taken, want, n = set(), [], 0
        while len(want) < S:
            r = inputs.splitmix64(seed, 2 * n, 2)
            x = int(inputs.bounded(r[0:1], W)[0])
            y = int(inputs.bounded(r[1:2], H)[0])
            n += 1
            if (x, y) not in taken:
                taken.add((x, y))
                want.append((x, y))
        assert np.array_equal(got, np.array(want, np.int32))


def test_place_seeds_distinct_in_range():
    xy = inputs.place_seeds(1000, 700, 5000, 9)
    assert xy[:, 0].min() >= 0 and xy[:, 0].max() < 1000
    assert xy[:, 1].min() >= 0 and xy[:, 1].max() < 700
    assert len(np.unique(xy[:, 1] * 1000 + xy[:, 0])) == 5000


def test_workload_recipes():
    assert inputs.small().sims[0].num_seeds == 256
    b = inputs.batched()
    assert len(b.sims) == 64
    assert all(s.width in (256, 512, 1024, 2048, 4096) for s in b.sims)
    assert all(64 <= s.num_seeds <= min(65536, s.width ** 2) for s in b.sims)
    v = inputs.serving()
    assert len(v.sims) == 256
    assert all(256 <= s.num_seeds <= min(1 << 18, s.width ** 2) for s in v.sims)
    t, tgt = inputs.poisson_arrivals(2000.0, 0.5, 256)
    assert 800 < len(t) < 1200 and (np.diff(t) > 0).all() and tgt.max() < 256


def test_band_recipe_is_one_eighth_of_the_large_grid(orc):
    """The band has the large workload's width, seed density, moves and
    first dJFA jump, and 1024 rows plus delta_1 halo rows on each side."""
    band, large = inputs.band().sims[0], inputs.large().sims[0]
    d1 = orc.delta1(large.width, large.height, large.num_seeds, 4)
    assert band.width == large.width and band.height == large.height // 8 + 2 * d1
    assert band.num_seeds * large.pixels == large.num_seeds * band.pixels
    assert (band.disp_lo, band.disp_hi) == (large.disp_lo, large.disp_hi)
    assert orc.delta1(band.width, band.height, band.num_seeds, 4) == d1 == 16
