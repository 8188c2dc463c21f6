"""Seeded synthetic inputs for Fourier ptychographic reconstruction.

This module is shared by the tests, the benchmark and the FP64 oracle's
harness.  It draws random numbers and shapes them into inputs -- tile
geometry, complex test objects, defocus distances, photon noise -- and holds
none of the reconstruction's arithmetic: no FFT, no spectrum crop, no
illumination-angle formula, no update rule.  Noise is applied to an
intensity stack that the caller computed with a forward model of its own.

Workloads stand in for the paper's experimental data (USAF chart and bee
wing, Sec. 4), which are not public; they follow the acquisition geometry of
Sec. 2.2 / Sec. 4 (LED board above the sample, per-sub-region illumination
angle and defocus, overlapping 2D tiles of the sensor, Sec. 3.1).

Seeding: ``numpy.random.SeedSequence(220302507).spawn(5)[w]`` is the root of
workload ``w`` (0 = single 64-px tile, 1 = full field of 16x16 tiles of
128 px, 2 = its precision variant, 3 = uneven batch, 4 = serving stream);
``.spawn(T)[t]`` is tile ``t``.  Each tile's generator draws, in order: the
amplitude Gaussians, the phase Gaussians, the defocus, then (at the caller's
request) the Poisson noise.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, asdict
from typing import List, Optional

import numpy as np

ROOT_SEED = 220302507

# Field names mirror ``fpm_tile_desc`` in include/fpm.h.
DESC_FIELDS = (
    "n", "upsample", "led_rows", "led_cols", "led_pitch_um", "led_height_um",
    "led_origin_x_um", "led_origin_y_um", "wavelength_um", "na_obj", "pixel_um",
    "tile_x_um", "tile_y_um", "defocus_um", "iterations", "pupil_update",
    "precision", "schedule",
)

SCHED_SEQUENTIAL = 0      # one LED at a time, ascending illumination NA
SCHED_LED_GROUPS = 1      # non-overlapping LED groups run concurrently
SCHED_GROUP_ORDER = 2     # one LED at a time, in the grouped sweep order
SCHED_PIPELINED = 3       # sequential sweep, updates of all iterations level-scheduled

PREC_FP32_FFT = 0
PREC_MFMA_BF16X3 = 1
PREC_MFMA_FP16 = 2


@dataclass
class TileDesc:
    """One tile = one independent reconstruction problem (Sec. 3.1)."""
    n: int
    upsample: int
    led_rows: int = 15
    led_cols: int = 15
    led_pitch_um: float = 4000.0
    led_height_um: float = 90000.0
    led_origin_x_um: float = 0.0
    led_origin_y_um: float = 0.0
    wavelength_um: float = 0.532
    na_obj: float = 0.1
    pixel_um: float = 1.625
    tile_x_um: float = 0.0
    tile_y_um: float = 0.0
    defocus_um: float = 0.0
    iterations: int = 10
    pupil_update: int = 1
    precision: int = PREC_FP32_FFT
    schedule: int = SCHED_SEQUENTIAL

    @property
    def N(self) -> int:
        return self.n * self.upsample

    @property
    def L(self) -> int:
        return self.led_rows * self.led_cols

    def as_dict(self):
        return asdict(self)


@dataclass
class TileDraw:
    """A tile's description plus its private random stream."""
    desc: TileDesc
    rng: np.random.Generator
    peak_photons: float = 1e4
    up_candidates: List[int] = field(default_factory=list)
    obj: Optional[np.ndarray] = None


def _root(workload: int) -> np.random.SeedSequence:
    return np.random.SeedSequence(ROOT_SEED).spawn(5)[workload]


def gaussian_field(rng: np.random.Generator, N: int, count: int = 20) -> np.ndarray:
    """Sum of ``count`` isotropic Gaussians on an N x N periodic grid.

    Centres U[0,N)^2, widths log-uniform in [1.5, N/8] pixels, weights U[0,1].
    Distances wrap around the grid so the field is periodic (no edge jump
    in its spectrum).  Returned in float64, not normalised.
    """
    centres = rng.uniform(0.0, N, size=(count, 2))
    sigmas = np.exp(rng.uniform(math.log(1.5), math.log(N / 8.0), size=count))
    weights = rng.uniform(0.0, 1.0, size=count)
    grid = np.arange(N, dtype=np.float64)
    out = np.zeros((N, N), dtype=np.float64)
    for (cy, cx), s, w in zip(centres, sigmas, weights):
        dy = np.abs(grid - cy)
        dy = np.minimum(dy, N - dy)
        dx = np.abs(grid - cx)
        dx = np.minimum(dx, N - dx)
        gy = np.exp(-0.5 * (dy / s) ** 2)
        gx = np.exp(-0.5 * (dx / s) ** 2)
        out += w * np.outer(gy, gx)
    return out


def _minmax(a: np.ndarray, lo: float, hi: float) -> np.ndarray:
    amin, amax = a.min(), a.max()
    if amax <= amin:
        return np.full_like(a, 0.5 * (lo + hi))
    return lo + (hi - lo) * (a - amin) / (amax - amin)


def random_object(rng: np.random.Generator, N: int) -> np.ndarray:
    """Complex128 N x N test object: amplitude in [0.5, 1], phase in [-pi/2, pi/2]."""
    amp = _minmax(gaussian_field(rng, N), 0.5, 1.0)
    phase = _minmax(gaussian_field(rng, N), -0.5 * math.pi, 0.5 * math.pi)
    return amp * np.exp(1j * phase)


def poisson_noise(rng: np.random.Generator, intensity: np.ndarray, peak: float) -> np.ndarray:
    """Shot noise at ``peak`` photons for the brightest pixel of the stack.

    I_meas = Poisson(c * I) / c with c = peak / max(I); returned as float32.
    Negative inputs (round-off of a forward model) are clipped to zero first.
    """
    I = np.maximum(np.asarray(intensity, dtype=np.float64), 0.0)
    m = I.max()
    if m <= 0:
        return I.astype(np.float32)
    c = peak / m
    return (rng.poisson(c * I) / c).astype(np.float32)


# ---------------------------------------------------------------- workloads

def single_tile_64(iterations: int = 10, schedule: int = SCHED_SEQUENTIAL,
                   pupil_update: int = 1) -> List[TileDraw]:
    """One 64-px tile, 15x15 LEDs (4 mm pitch, 90 mm high), 4x upsampling."""
    ss = _root(0).spawn(1)[0]
    rng = np.random.default_rng(ss)
    d = TileDesc(n=64, upsample=4, iterations=iterations, schedule=schedule,
                 pupil_update=pupil_update)
    return [TileDraw(desc=d, rng=rng, peak_photons=1e4)]


def full_fov_tiles(tiles_per_side: int = 16, n: int = 128, overlap: int = 8,
                   sensor: int = 2048, iterations: int = 20,
                   schedule: int = SCHED_LED_GROUPS, pupil_update: int = 1,
                   workload: int = 1, only: Optional[List[int]] = None) -> List[TileDraw]:
    """A 2048-px sensor cut into 16x16 overlapping 128-px tiles.

    Stride n - overlap = 120; the tile grid (1928 px) is centred on the
    sensor, so tile (ty, tx) starts at pixel 60 + 120*t on each axis and its
    centre sits (60 + 120 t + 64 - 1024) pixels from the optical axis.
    Each tile draws its own object and a defocus z ~ U[-20, 20] um.
    ``only`` restricts the draw to the listed tile indices (the streams of
    the others are still spawned, so a tile's inputs do not depend on it).
    """
    T = tiles_per_side * tiles_per_side
    stride = n - overlap
    span = stride * (tiles_per_side - 1) + n
    first = (sensor - span) // 2
    seeds = _root(workload).spawn(T)
    out = []
    for t in range(T):
        if only is not None and t not in only:
            continue
        ty, tx = divmod(t, tiles_per_side)
        rng = np.random.default_rng(seeds[t])
        d = TileDesc(n=n, upsample=4, iterations=iterations, schedule=schedule,
                     pupil_update=pupil_update)
        pix = 1.625
        d.tile_x_um = (first + stride * tx + n / 2 - sensor / 2) * pix
        d.tile_y_um = (first + stride * ty + n / 2 - sensor / 2) * pix
        out.append(TileDraw(desc=d, rng=rng, peak_photons=1e4))
    return out


def uneven_batch(T: int = 512, only: Optional[List[int]] = None,
                 schedule: int = SCHED_LED_GROUPS, workload: int = 3,
                 sizes=(64, 96, 128, 256), grids=(9, 13, 15, 21)) -> List[TileDraw]:
    """Uneven tiles: n, LED grid, upsampling, defocus, photons and iteration
    count drawn per tile.  ``up_candidates`` is a random permutation of
    {3, 4, 5}; the consumer takes the first value whose crop windows stay
    inside the high-resolution grid (a geometry check that belongs to the
    planner, not to this module)."""
    seeds = _root(workload).spawn(T)
    out = []
    for t in range(T):
        if only is not None and t not in only:
            continue
        rng = np.random.default_rng(seeds[t])
        n = int(rng.choice(sizes))
        g = int(rng.choice(grids))
        ups = [int(u) for u in rng.permutation([3, 4, 5])]
        z = float(rng.uniform(-30.0, 30.0))
        peak = float(math.exp(rng.uniform(math.log(1e3), math.log(1e5))))
        iters = int(rng.integers(5, 31))
        tx, ty = (float(v) for v in rng.uniform(-1500.0, 1500.0, size=2))
        d = TileDesc(n=n, upsample=ups[0], led_rows=g, led_cols=g, iterations=iters,
                     schedule=schedule, tile_x_um=tx, tile_y_um=ty, defocus_um=z)
        out.append(TileDraw(desc=d, rng=rng, peak_photons=peak, up_candidates=ups))
    return out


def draw_object_and_defocus(td: TileDraw, z_range: Optional[float] = None) -> np.ndarray:
    """Draw this tile's object (and, if ``z_range`` is given, its defocus
    z ~ U[-z_range, z_range]) from the tile's stream, in that order."""
    td.obj = random_object(td.rng, td.desc.N)
    if z_range is not None:
        td.desc.defocus_um = float(td.rng.uniform(-z_range, z_range))
    return td.obj


def shared_object_tiles(tiles_per_side: int = 3, n: int = 64, overlap: int = 8,
                        upsample: int = 4, iterations: int = 8,
                        schedule: int = SCHED_LED_GROUPS, pupil_update: int = 0,
                        workload: int = 1):
    """Tiles cut from ONE object (the synthetic stand-in for the paper's
    bee-wing field of Sec. 4.2): a (tiles_per_side)^2 grid of n-px tiles with
    `overlap` LR pixels between neighbours (0: abutting tiles), each tile at
    its own position under the LED array.  Returns (tile draws, the whole
    high-resolution object, HR stride).  The object is drawn once from the
    workload's first stream; tile t's draws use its own spawned stream."""
    stride = n - overlap
    span = stride * (tiles_per_side - 1) + n
    ss = _root(workload).spawn(2)
    rng0 = np.random.default_rng(ss[0])
    whole = random_object(rng0, upsample * span)
    seeds = ss[1].spawn(tiles_per_side * tiles_per_side)
    out = []
    pix = 1.625
    for t in range(tiles_per_side * tiles_per_side):
        ty, tx = divmod(t, tiles_per_side)
        d = TileDesc(n=n, upsample=upsample, iterations=iterations, schedule=schedule,
                     pupil_update=pupil_update)
        d.tile_x_um = (stride * tx + n / 2 - span / 2) * pix
        d.tile_y_um = (stride * ty + n / 2 - span / 2) * pix
        td = TileDraw(desc=d, rng=np.random.default_rng(seeds[t]), peak_photons=1e4)
        hs = upsample * stride
        td.obj = whole[ty * hs:ty * hs + upsample * n, tx * hs:tx * hs + upsample * n].copy()
        out.append(td)
    return out, whole, upsample * stride
