"""FP64 CPU oracle for Fourier ptychographic reconstruction -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never calls it and
shares no code with it.  The arithmetic lives in ``fpm_oracle.c`` (plain C,
double precision); this module builds it with gcc and marshals numpy arrays.

Functions whose results are pinned by the CPU tests against values fixed by
the mathematics (brute-force DFT, closed forms, invariants) are listed in the
test-suite; see ``tests/test_oracle_pins.py``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fpm_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

SEQUENTIAL, LED_GROUPS, GROUP_ORDER = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-shared", "-fPIC", "-fopenmp",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class Geom(C.Structure):
    _fields_ = [
        ("n", C.c_int32), ("up", C.c_int32),
        ("led_rows", C.c_int32), ("led_cols", C.c_int32),
        ("led_pitch_um", C.c_double), ("led_height_um", C.c_double),
        ("led_x0_um", C.c_double), ("led_y0_um", C.c_double),
        ("wavelength_um", C.c_double), ("na", C.c_double), ("pixel_um", C.c_double),
        ("tile_x_um", C.c_double), ("tile_y_um", C.c_double),
        ("defocus_um", C.c_double),
    ]


def geom(desc) -> Geom:
    """Build the oracle's geometry record from a TileDesc-like object."""
    g = Geom()
    g.n, g.up = desc.n, desc.upsample
    g.led_rows, g.led_cols = desc.led_rows, desc.led_cols
    g.led_pitch_um, g.led_height_um = desc.led_pitch_um, desc.led_height_um
    g.led_x0_um, g.led_y0_um = desc.led_origin_x_um, desc.led_origin_y_um
    g.wavelength_um, g.na, g.pixel_um = desc.wavelength_um, desc.na_obj, desc.pixel_um
    g.tile_x_um, g.tile_y_um = desc.tile_x_um, desc.tile_y_um
    g.defocus_um = desc.defocus_um
    return g


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        L = C.CDLL(_LIB_PATH)
        dp, fp, ip, up8 = (C.POINTER(C.c_double), C.POINTER(C.c_float),
                           C.POINTER(C.c_int32), C.POINTER(C.c_uint8))
        gp = C.POINTER(Geom)
        L.orc_fft1.argtypes = [dp, C.c_int32, C.c_int32]
        L.orc_fft2.argtypes = [dp, C.c_int32, C.c_int32, C.c_int32]
        L.orc_set_threads.argtypes = [C.c_int32]
        L.orc_support.argtypes = [gp, up8]
        L.orc_support.restype = C.c_int32
        L.orc_pupil_init.argtypes = [gp, dp]
        L.orc_offsets.argtypes = [gp, ip]
        L.orc_offsets.restype = C.c_int32
        L.orc_order.argtypes = [gp, ip]
        L.orc_groups.argtypes = [gp, ip, ip, ip, ip, ip]
        L.orc_groups.restype = C.c_int32
        L.orc_object_to_spectrum.argtypes = [gp, dp, dp]
        L.orc_spectrum_to_object.argtypes = [gp, dp, dp]
        L.orc_forward.argtypes = [gp, dp, dp, dp]
        L.orc_reconstruct.argtypes = [gp, fp, C.c_int32, C.c_int32, C.c_int32,
                                      dp, dp, dp, dp, dp]
        L.orc_reconstruct.restype = C.c_int32
        L.orc_reconstruct_online.argtypes = [gp, fp, C.c_int32, C.c_int32, ip, dp, dp, dp]
        L.orc_reconstruct_online.restype = C.c_int32
        _lib = L
    return _lib


def set_threads(k: int) -> None:
    """Threads for the oracle's line transforms (results do not depend on it)."""
    lib().orc_set_threads(int(k))


def _p(a, t):
    return a.ctypes.data_as(C.POINTER(t))


def _c128(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


def fft1(z, inverse=False):
    z = _c128(z).copy()
    lib().orc_fft1(_p(z, C.c_double), z.shape[0], 1 if inverse else -1)
    return z


def fft2(z, inverse=False):
    z = _c128(z).copy()
    lib().orc_fft2(_p(z, C.c_double), z.shape[0], z.shape[1], 1 if inverse else -1)
    return z


def support(desc):
    g = geom(desc)
    m = np.zeros((desc.n, desc.n), dtype=np.uint8)
    cnt = lib().orc_support(C.byref(g), _p(m, C.c_uint8))
    return m.astype(bool), int(cnt)


def pupil_init(desc):
    g = geom(desc)
    P = np.zeros((desc.n, desc.n), dtype=np.complex128)
    lib().orc_pupil_init(C.byref(g), _p(P, C.c_double))
    return P


def offsets(desc):
    """(status, int32 [L][2] (drow, dcol)) in grid LED order."""
    g = geom(desc)
    off = np.zeros((desc.led_rows * desc.led_cols, 2), dtype=np.int32)
    st = lib().orc_offsets(C.byref(g), _p(off, C.c_int32))
    return int(st), off


def order(desc):
    g = geom(desc)
    o = np.zeros(desc.led_rows * desc.led_cols, dtype=np.int32)
    lib().orc_order(C.byref(g), _p(o, C.c_int32))
    return o


@dataclass
class Groups:
    group_of: np.ndarray
    sweep: np.ndarray
    gstart: np.ndarray
    count: int


def groups(desc):
    g = geom(desc)
    L = desc.led_rows * desc.led_cols
    _, off = offsets(desc)
    o = order(desc)
    gof = np.zeros(L, dtype=np.int32)
    sw = np.zeros(L, dtype=np.int32)
    gs = np.zeros(L + 1, dtype=np.int32)
    ng = lib().orc_groups(C.byref(g), _p(off, C.c_int32), _p(o, C.c_int32),
                          _p(gof, C.c_int32), _p(sw, C.c_int32), _p(gs, C.c_int32))
    return Groups(gof, sw, gs[:ng + 1].copy(), int(ng))


def object_to_spectrum(desc, obj):
    g = geom(desc)
    o = _c128(obj)
    S = np.zeros_like(o)
    lib().orc_object_to_spectrum(C.byref(g), _p(o, C.c_double), _p(S, C.c_double))
    return S


def spectrum_to_object(desc, S):
    g = geom(desc)
    S = _c128(S)
    o = np.zeros_like(S)
    lib().orc_spectrum_to_object(C.byref(g), _p(S, C.c_double), _p(o, C.c_double))
    return o


def forward(desc, S, P=None):
    """Low-resolution intensities [L][n][n] (float64) from spectrum S and pupil P."""
    g = geom(desc)
    S = _c128(S)
    P = pupil_init(desc) if P is None else _c128(P)
    I = np.zeros((desc.led_rows * desc.led_cols, desc.n, desc.n), dtype=np.float64)
    lib().orc_forward(C.byref(g), _p(S, C.c_double), _p(P, C.c_double), _p(I, C.c_double))
    return I


@dataclass
class Result:
    S: np.ndarray
    P: np.ndarray
    residual: np.ndarray
    status: int


def reconstruct(desc, I, iterations=None, pupil_update=None, schedule=None,
                S_in=None, P_in=None) -> Result:
    g = geom(desc)
    iters = desc.iterations if iterations is None else iterations
    pu = desc.pupil_update if pupil_update is None else pupil_update
    sc = desc.schedule if schedule is None else schedule
    I = np.ascontiguousarray(I, dtype=np.float32)
    N = desc.n * desc.upsample
    S = np.zeros((N, N), dtype=np.complex128)
    P = np.zeros((desc.n, desc.n), dtype=np.complex128)
    res = np.zeros(max(iters, 1), dtype=np.float64)
    Sin = None if S_in is None else _c128(S_in)
    Pin = None if P_in is None else _c128(P_in)
    st = lib().orc_reconstruct(
        C.byref(g), _p(I, C.c_float), iters, pu, sc,
        None if Sin is None else _p(Sin, C.c_double),
        None if Pin is None else _p(Pin, C.c_double),
        _p(S, C.c_double), _p(P, C.c_double), _p(res, C.c_double))
    return Result(S, P, res[:iters], int(st))


def reconstruct_online(desc, I, arrival, iterations=None, pupil_update=None) -> Result:
    """Sec. 3.4 Fig. 7a: the sequential reconstruction with the images
    arriving in `arrival` (grid LED indices); see orc_reconstruct_online."""
    g = geom(desc)
    iters = desc.iterations if iterations is None else iterations
    pu = desc.pupil_update if pupil_update is None else pupil_update
    I = np.ascontiguousarray(I, dtype=np.float32)
    arr = np.ascontiguousarray(arrival, dtype=np.int32)
    if arr.size != desc.led_rows * desc.led_cols:
        raise ValueError("arrival must list every LED once")
    N = desc.n * desc.upsample
    S = np.zeros((N, N), dtype=np.complex128)
    P = np.zeros((desc.n, desc.n), dtype=np.complex128)
    res = np.zeros(max(iters, 1), dtype=np.float64)
    st = lib().orc_reconstruct_online(C.byref(g), _p(I, C.c_float), iters, pu,
                                      _p(arr, C.c_int32), _p(S, C.c_double),
                                      _p(P, C.c_double), _p(res, C.c_double))
    return Result(S, P, res[:iters], int(st))


def object_from_result(desc, r: Result):
    return spectrum_to_object(desc, r.S)


def synthesize(td, z_range=None, noise=True, peak=None):
    """Draw a tile's object (and defocus) from its stream, then its intensity
    stack with this oracle's FP64 forward model and the stream's shot noise.
    Returns (object, true pupil, float32 intensities)."""
    import fpm_synth
    obj = fpm_synth.draw_object_and_defocus(td, z_range)
    S = object_to_spectrum(td.desc, obj)
    P = pupil_init(td.desc)
    I = forward(td.desc, S, P)
    if noise:
        I = fpm_synth.poisson_noise(td.rng, I, td.peak_photons if peak is None else peak)
    else:
        I = I.astype(np.float32)
    return obj, P, I
