"""FP64 stitching of reconstructed tiles -- TEST INFRASTRUCTURE (the oracle).

Sec. 3.1, Eq. (1): two overlapping complex sub-images f1 and f2 become one
image f that takes f1 up to the middle of their overlap and (mu1 / mu2) * f2
after it, mu1 and mu2 being complex means; a row of tiles is merged left to
right ("part 1", along x), then the merged rows top to bottom ("part 2",
along y).  Readings where the paper is silent:
  * mu1, mu2 are the means of f1 and f2 over their shared overlap strip
    (the only pixels both images cover, which is what the ratio is for: it
    undoes each tile's own global complex factor);
  * "middle" is width - overlap // 2 in f1's coordinates;
  * with no overlap the ratio is 1 (plain concatenation).
Plain numpy in complex128, written from the equation; shares nothing with the
GPU library.  Only tests/ and bench.py use it.
"""
from __future__ import annotations

import numpy as np


def stitch_pair(f1: np.ndarray, f2: np.ndarray, overlap: int, axis: int = 1) -> np.ndarray:
    """Eq. (1) for two images sharing `overlap` pixels along `axis` (1: x,
    f2 to the right of f1; 0: y, f2 below f1)."""
    f1 = np.asarray(f1, dtype=np.complex128)
    f2 = np.asarray(f2, dtype=np.complex128)
    if axis == 0:
        return stitch_pair(f1.T, f2.T, overlap, axis=1).T
    rows, w1 = f1.shape
    w2 = f2.shape[1]
    assert f2.shape[0] == rows and 0 <= overlap <= min(w1, w2)
    if overlap > 0:
        mu1 = f1[:, w1 - overlap:].mean()
        mu2 = f2[:, :overlap].mean()
        ratio = mu1 / mu2
    else:
        ratio = 1.0
    out = np.empty((rows, w1 + w2 - overlap), dtype=np.complex128)
    cut = w1 - overlap // 2                      # x < cut: f1
    out[:, :cut] = f1[:, :cut]
    out[:, cut:] = ratio * f2[:, cut - (w1 - overlap):]
    return out


def stitch_grid(tiles, overlap: int) -> np.ndarray:
    """tiles[r][c]: equal-size complex images on a grid whose neighbours share
    `overlap` pixels; rows are merged along x first, then along y."""
    strips = []
    for row in tiles:
        s = np.asarray(row[0], dtype=np.complex128)
        for t in row[1:]:
            s = stitch_pair(s, t, overlap, axis=1)
        strips.append(s)
    out = strips[0]
    for s in strips[1:]:
        out = stitch_pair(out, s, overlap, axis=0)
    return out
