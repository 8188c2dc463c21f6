"""FP64 defocus-distance estimation of one sub-region -- TEST INFRASTRUCTURE
(the oracle).  Only tests/, __graft_entry__.smoke() and bench.py's CPU
baseline use it; it shares nothing with the GPU library.

The paper estimates each sub-region's defocus distance before its
reconstruction, offline, from at least nine bright-field images (Sec. 3.4,
Fig. 7b; the sub-regions' own defocus, Sec. 2.2).  The algorithm it cites is
not in the text, so this is a reading written from the method itself:

* The bright-field LEDs of a tile are those whose illumination falls inside
  the objective's aperture: the window's zero-frequency bin, at
  (n/2 - drow, n/2 - dcol) in the window, lies in the support disc D0,
  i.e. drow^2 + dcol^2 <= r^2 with r = NA n dx / lambda (integer offsets of
  Sec. 2.2).  At least nine are required.
* The search runs on the smallest centred block of the LED grid that holds
  every bright-field LED (an odd block for an odd grid, an even one for an
  even grid, rows and columns apart): the same LEDs at the same positions,
  with the block's images.
* For each candidate z on the grid z_lo, z_lo + step, ... <= z_hi, the
  block is reconstructed with the pupil fixed at the defocus pupil of z
  (P = D0 H_z, no pupil recovery), LED groups, `iterations` iterations from
  the usual initial guess; its score is the residual of the last iteration.
  The right pupil makes the images most consistent with one spectrum, so the
  score is least near the true z.
* z is the vertex of the parabola through the smallest score and its two
  neighbours (the grid point itself at either end of the grid, or where the
  three points are not convex).
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass
from typing import List

import numpy as np

from . import LED_GROUPS, offsets, reconstruct

MIN_BRIGHT_FIELD = 9


@dataclass
class DefocusResult:
    z_um: float              # estimated defocus distance
    candidates: np.ndarray   # candidate z values
    scores: np.ndarray       # last-iteration residual per candidate
    best: int                # index of the smallest score
    bright_field: List[int]  # grid indices of the tile's bright-field LEDs
    block: tuple             # (row0, col0, rows, cols) of the LED block searched


def bright_field_leds(desc) -> List[int]:
    """Grid indices of the LEDs whose zero-frequency bin falls in D0."""
    st, off = offsets(desc)
    if st != 0:
        raise ValueError("geometry rejected by the plan's window bound")
    r = desc.na_obj * desc.n * desc.pixel_um / desc.wavelength_um
    return [j for j in range(desc.led_rows * desc.led_cols)
            if int(off[j][0]) ** 2 + int(off[j][1]) ** 2 <= r * r]


def _centred_span(total: int, used: List[int]) -> tuple:
    """Smallest centred run [start, start + m) of 0..total-1, m of the same
    parity as total, that contains every index in `used`."""
    for m in range(2 - total % 2, total + 1, 2):
        start = (total - m) // 2
        if all(start <= u < start + m for u in used):
            return start, m
    return 0, total


def search_block(desc):
    """(row0, col0, rows, cols, bright-field LEDs) of the LED block the
    search runs on."""
    bf = bright_field_leds(desc)
    if len(bf) < MIN_BRIGHT_FIELD:
        raise ValueError(f"{len(bf)} bright-field LEDs; the estimate needs at least "
                         f"{MIN_BRIGHT_FIELD}")
    r0, mr = _centred_span(desc.led_rows, [j // desc.led_cols for j in bf])
    c0, mc = _centred_span(desc.led_cols, [j % desc.led_cols for j in bf])
    return r0, c0, mr, mc, bf


def candidates(z_lo: float, z_hi: float, step: float) -> np.ndarray:
    """z_lo, z_lo + step, ... up to z_hi (inclusive within step/1e6)."""
    if not (step > 0 and z_hi >= z_lo):
        raise ValueError("need step > 0 and z_hi >= z_lo")
    k = int(np.floor((z_hi - z_lo) / step + 1e-6)) + 1
    return z_lo + step * np.arange(k, dtype=np.float64)


def parabola_vertex(zs: np.ndarray, scores: np.ndarray, best: int) -> float:
    """Vertex of the parabola through (z, score) at best-1, best, best+1 on
    the uniform grid zs; zs[best] at the grid's ends or without convexity."""
    if best <= 0 or best >= len(zs) - 1:
        return float(zs[best])
    a, b, c = float(scores[best - 1]), float(scores[best]), float(scores[best + 1])
    curv = a - 2.0 * b + c
    if not curv > 0.0:
        return float(zs[best])
    step = float(zs[1] - zs[0])
    return float(zs[best]) + 0.5 * step * (a - c) / curv


def estimate_defocus(desc, I, z_lo: float = -40.0, z_hi: float = 40.0, step: float = 5.0,
                     iterations: int = 10) -> DefocusResult:
    """The defocus distance of the tile `desc` (its own defocus_um is not
    used) from its intensity stack I [L][n][n] (grid order)."""
    I = np.asarray(I, dtype=np.float32).reshape(desc.led_rows * desc.led_cols, desc.n, desc.n)
    r0, c0, mr, mc, bf = search_block(desc)
    idx = [(r0 + r) * desc.led_cols + c0 + c for r in range(mr) for c in range(mc)]
    I_blk = np.ascontiguousarray(I[idx])
    zs = candidates(z_lo, z_hi, step)
    scores = np.empty(len(zs))
    for k, z in enumerate(zs):
        d = dataclasses.replace(desc, led_rows=mr, led_cols=mc, defocus_um=float(z),
                                iterations=iterations, pupil_update=0, schedule=LED_GROUPS)
        res = reconstruct(d, I_blk)
        if res.status != 0:
            raise RuntimeError(f"reconstruction at z = {z} failed ({res.status})")
        scores[k] = res.residual[-1]
    best = int(np.argmin(scores))
    return DefocusResult(z_um=parabola_vertex(zs, scores, best), candidates=zs, scores=scores,
                         best=best, bright_field=bf, block=(r0, c0, mr, mc))
