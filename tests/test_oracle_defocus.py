"""Pins of the oracle's defocus-distance estimate (Sec. 3.4 Fig. 7b: the
sub-region's defocus from its bright-field images before reconstruction;
Sec. 2.2: each sub-region has its own defocus).  Each pin checks the
estimate against something other than itself: the known z the synthetic
data were made with, brute-force geometry, the closed-form vertex of a
parabola, and the in-focus case."""
import dataclasses

import numpy as np
import pytest

import fpm_synth
from oracle import defocus as odf

pytestmark = pytest.mark.filterwarnings("ignore")


def tile(z, n=64, x=0.0, y=0.0, rows=15, seed=0):
    d = fpm_synth.TileDesc(n=n, upsample=4, led_rows=rows, led_cols=rows, iterations=1,
                           defocus_um=z, tile_x_um=x, tile_y_um=y)
    return d, fpm_synth.TileDraw(desc=d, rng=np.random.default_rng(seed))


def test_parabola_vertex_is_exact_for_a_parabola():
    zs = np.arange(-20.0, 21.0, 5.0)
    for z0 in (-7.3, 0.0, 2.4, 12.9):
        scores = 0.3 + 1.7 * (zs - z0) ** 2
        best = int(np.argmin(scores))
        assert abs(odf.parabola_vertex(zs, scores, best) - z0) < 1e-9
    # at the grid's end, or without convexity: the grid point itself
    scores = (zs - 30.0) ** 2
    assert odf.parabola_vertex(zs, scores, len(zs) - 1) == zs[-1]
    flat = np.ones_like(zs)
    assert odf.parabola_vertex(zs, flat, 3) == zs[3]


def test_bright_field_set_matches_a_brute_force_aperture_test(orc):
    """An LED is bright-field iff its window's zero-frequency bin lies in the
    support disc: checked on the disc mask itself, bin by bin."""
    for x, y in ((0.0, 0.0), (900.0, -400.0), (-1500.0, 1500.0)):
        d, _ = tile(0.0, x=x, y=y)
        mask, _ = orc.support(d)
        st, off = orc.offsets(d)
        n = d.n
        brute = [j for j in range(d.L)
                 if 0 <= n // 2 - off[j][0] < n and 0 <= n // 2 - off[j][1] < n
                 and mask[n // 2 - off[j][0], n // 2 - off[j][1]]]
        assert odf.bright_field_leds(d) == brute
        assert len(brute) >= 9


def test_search_block_is_the_smallest_centred_block_holding_the_bright_field():
    d, _ = tile(0.0, x=1200.0, y=-700.0)
    r0, c0, mr, mc, bf = odf.search_block(d)
    assert mr % 2 == d.led_rows % 2 and mc % 2 == d.led_cols % 2
    assert r0 == (d.led_rows - mr) // 2 and c0 == (d.led_cols - mc) // 2
    rows = [j // d.led_cols for j in bf]
    cols = [j % d.led_cols for j in bf]
    assert r0 <= min(rows) and max(rows) < r0 + mr
    assert c0 <= min(cols) and max(cols) < c0 + mc
    # two fewer rows (or columns) would drop a bright-field LED
    assert mr == 1 or not (r0 + 1 <= min(rows) and max(rows) < r0 + mr - 1)
    assert mc == 1 or not (c0 + 1 <= min(cols) and max(cols) < c0 + mc - 1)


def test_too_few_bright_field_images_are_rejected():
    # a 3x3 board leaves at most nine LEDs, and a wide pitch pushes all but
    # the centre one out of the aperture
    d = fpm_synth.TileDesc(n=64, upsample=4, led_rows=3, led_cols=3, led_pitch_um=12000.0,
                           iterations=1)
    with pytest.raises(ValueError):
        odf.search_block(d)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_recovers_the_known_defocus_of_synthetic_tiles(orc, seed):
    """Noisy stacks (1e4 peak photons) made with a known z at random tile
    positions: the estimate lands within 0.5 um of it."""
    rng = np.random.default_rng(100 + seed)
    z = float(rng.uniform(-30.0, 30.0))
    d, td = tile(z, x=float(rng.uniform(-1000, 1000)), y=float(rng.uniform(-1000, 1000)),
                 seed=seed)
    _, _, I = orc.synthesize(td)
    d_blind = dataclasses.replace(d, defocus_um=0.0)
    r = odf.estimate_defocus(d_blind, I)
    print(f"z {z:+.3f} estimate {r.z_um:+.3f}")
    assert abs(r.z_um - z) < 0.5
    assert abs(r.candidates[r.best] - z) <= 2.5 + 1e-9   # the best grid point is the nearest


def test_in_focus_tile_gives_zero(orc):
    """Noiseless data of an in-focus tile: the grid point z = 0 scores best
    and the refined estimate stays within 0.3 um of it."""
    d, td = tile(0.0, seed=4)
    _, _, I = orc.synthesize(td, noise=False)
    r = odf.estimate_defocus(d, I, z_lo=-20.0, z_hi=20.0, step=5.0)
    assert abs(r.z_um) < 0.3
    assert r.candidates[r.best] == 0.0


def test_candidate_grid():
    assert np.allclose(odf.candidates(-10, 10, 5), [-10, -5, 0, 5, 10])
    assert np.allclose(odf.candidates(0, 9.9, 5), [0, 5])
    with pytest.raises(ValueError):
        odf.candidates(0, 10, 0)
