"""Pins of the stitching oracle (Sec. 3.1, Eq. (1)) against values the paper
prints and properties the equation fixes: the stitched size of the paper's
example, exact reassembly of consistent tiles that carry unknown global
complex factors (what the mu1/mu2 weight is for), which image owns each side
of the overlap's middle, plain concatenation without overlap, and the x/y
symmetry of the two parts."""
import os

import numpy as np
import pytest

from oracle import stitch as st

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "stitch_sizes.txt")


def rand_c(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def test_paper_example_size():
    rows = [r for r in open(GOLDEN) if r.strip() and not r.startswith("#")]
    assert rows
    for r in rows:
        w1, w2, h, ov, want = (int(v) for v in r.split())
        rng = np.random.default_rng(w1 + ov)
        out = st.stitch_pair(rand_c(rng, (h, w1)), rand_c(rng, (h, w2)), ov, axis=1)
        assert out.shape == (h, want)
        # part 2 on the transposed pair gives the transposed size
        outy = st.stitch_pair(rand_c(rng, (w1, h)), rand_c(rng, (w2, h)), ov, axis=0)
        assert outy.shape == (want, h)


@pytest.mark.parametrize("grid,side,ov", [((1, 2), 40, 6), ((3, 1), 32, 8), ((3, 4), 48, 10),
                                          ((4, 4), 64, 16)])
def test_consistent_tiles_with_global_factors_reassemble_exactly(grid, side, ov):
    """Tiles cut from one complex image, each multiplied by its own unknown
    complex factor (the global phase/scale freedom of every reconstruction):
    the stitched result is the image times the first tile's factor."""
    R, Cc = grid
    rng = np.random.default_rng(R * 100 + Cc)
    s = side - ov
    H, W = R * s + ov, Cc * s + ov
    img = rand_c(rng, (H, W)) + 3.0
    fac = np.exp(1j * rng.uniform(-np.pi, np.pi, (R, Cc))) * rng.uniform(0.5, 2.0, (R, Cc))
    tiles = [[fac[r, c] * img[r * s:r * s + side, c * s:c * s + side] for c in range(Cc)]
             for r in range(R)]
    out = st.stitch_grid(tiles, ov)
    assert out.shape == (H, W)
    ref = fac[0, 0] * img
    assert np.abs(out - ref).max() <= 1e-12 * np.abs(ref).max()


def test_overlap_middle_decides_the_owner():
    """A defect in f1's copy of the overlap shows up in the result only on
    f1's side of the overlap's middle; a defect in f2's copy only on f2's."""
    rng = np.random.default_rng(5)
    h, w, ov = 12, 30, 8
    img = rand_c(rng, (h, 2 * w - ov)) + 4.0
    f1, f2 = img[:, :w].copy(), img[:, w - ov:].copy()
    mid = w - ov // 2
    d1, d2 = f1.copy(), f2.copy()
    d1[:, mid - 1] += 100.0            # last column f1 keeps
    d1[:, mid] += 100.0                # first column f2 takes over
    out = st.stitch_pair(d1, f2, ov)
    # the defects shift mu1 a little; compare with the equation's own ratio
    ratio = d1[:, w - ov:].mean() / f2[:, :ov].mean()
    assert np.allclose(out[:, mid - 1], d1[:, mid - 1])
    assert np.allclose(out[:, mid], ratio * f2[:, ov // 2])
    d2[:, ov // 2 - 1] += 100.0        # f2's copy of f1's side: dropped
    out = st.stitch_pair(f1, d2, ov)
    assert np.allclose(out[:, :mid], f1[:, :mid])


def test_zero_overlap_concatenates():
    rng = np.random.default_rng(9)
    tiles = [[rand_c(rng, (5, 7)) for _ in range(3)] for _ in range(2)]
    out = st.stitch_grid(tiles, 0)
    assert np.array_equal(out, np.block(tiles))


def test_parts_are_transposes():
    rng = np.random.default_rng(11)
    a, b = rand_c(rng, (20, 16)), rand_c(rng, (20, 16))
    assert np.allclose(st.stitch_pair(a, b, 6, axis=1),
                       st.stitch_pair(a.T, b.T, 6, axis=0).T, rtol=0, atol=0)
