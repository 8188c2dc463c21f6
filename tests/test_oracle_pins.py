"""Pins for the FP64 oracle: each test checks the oracle against something
other than itself -- brute-force sums, closed forms, invariants, special cases
that reduce to a textbook routine -- so that a dropped term, a wrong sign or
index, or a transposed operand in the oracle fails at least one of them."""
import math

import numpy as np
import pytest

import fpm_synth
from fpm_synth import TileDesc


def tiny(n=16, up=2, grid=5, z=0.0, na=0.1, tile=(0.0, 0.0), pitch=4000.0):
    return TileDesc(n=n, upsample=up, led_rows=grid, led_cols=grid, led_pitch_um=pitch,
                    defocus_um=z, na_obj=na, tile_x_um=tile[0], tile_y_um=tile[1],
                    iterations=3)


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


# ------------------------------------------------------------------ FFT pins

def brute_dft(x, inverse=False):
    """O(n^2) DFT straight from the definition, no FFT library involved."""
    n = x.shape[0]
    j = np.arange(n)
    sgn = 1.0 if inverse else -1.0
    W = np.exp(sgn * 2j * np.pi * np.outer(j, j) / n)
    y = W @ x
    return y / n if inverse else y


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 7, 8, 12, 15, 16, 24, 32, 96])
def test_fft1_matches_bruteforce_dft(orc, n):
    rng = np.random.default_rng(n)
    x = rng.normal(size=n) + 1j * rng.normal(size=n)
    assert rel(orc.fft1(x), brute_dft(x)) < 1e-12
    assert rel(orc.fft1(x, inverse=True), brute_dft(x, inverse=True)) < 1e-12


@pytest.mark.parametrize("shape", [(4, 6), (8, 8), (12, 5), (16, 32), (3, 10)])
def test_fft2_matches_separable_bruteforce(orc, shape):
    rng = np.random.default_rng(sum(shape))
    x = rng.normal(size=shape) + 1j * rng.normal(size=shape)
    ref = np.stack([brute_dft(c) for c in x.T], axis=1)
    ref = np.stack([brute_dft(r) for r in ref], axis=0)
    assert rel(orc.fft2(x), ref) < 1e-12
    # library routine as a second, unrelated check
    assert rel(orc.fft2(x), np.fft.fft2(x)) < 1e-12


def test_fft_parseval_inverse_impulse_planewave(orc):
    rng = np.random.default_rng(7)
    n = 64
    x = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    X = orc.fft2(x)
    assert abs(np.sum(abs(X) ** 2) / n ** 2 - np.sum(abs(x) ** 2)) < 1e-9 * np.sum(abs(x) ** 2)
    assert rel(orc.fft2(X, inverse=True), x) < 1e-13
    d = np.zeros((n, n), complex)
    d[0, 0] = 1.0
    assert np.allclose(orc.fft2(d), 1.0, atol=1e-14)
    yy, xx = np.mgrid[0:n, 0:n]
    pw = np.exp(2j * np.pi * (3 * yy + 5 * xx) / n)
    F = orc.fft2(pw)
    assert abs(F[3, 5] - n * n) < 1e-9
    F[3, 5] = 0
    assert np.abs(F).max() < 1e-9


# --------------------------------------------------------- support / pupil

def lattice_disc_count(r, n):
    """Closed-form lattice count of the disc: sum over rows of chord widths."""
    cnt = 0
    for a in range(-n // 2, n // 2):
        if a * a <= r * r:
            w = int(math.isqrt(int(math.floor(r * r - a * a))))
            lo, hi = max(-w, -n // 2), min(w, n // 2 - 1)
            cnt += hi - lo + 1
    return cnt


@pytest.mark.parametrize("n,na", [(16, 0.1), (64, 0.1), (96, 0.1), (128, 0.1), (32, 0.05)])
def test_support_count_closed_form(orc, n, na):
    d = tiny(n=n, na=na)
    mask, cnt = orc.support(d)
    r = na * n * d.pixel_um / d.wavelength_um
    assert cnt == lattice_disc_count(r, n) == mask.sum()
    # known counts for the 15x15 workloads (lattice points within r)
    if n == 64 and na == 0.1:
        assert cnt == 1201
    if n == 128 and na == 0.1:
        assert cnt == 4809


def test_cutoff_passes_below_blocks_above(orc):
    """Sec. 2.1: the objective is a circular low-pass of cutoff NA/lambda.  A
    plane-wave object under the on-axis LED is imaged at unit intensity if
    its spatial frequency is below the cutoff and vanishes above it."""
    d = TileDesc(n=32, upsample=2, led_rows=1, led_cols=1)
    N = d.N
    fc = d.na_obj / d.wavelength_um              # cycles / um
    dxh = d.pixel_um / d.upsample                # HR pixel
    yy, xx = np.mgrid[0:N, 0:N]
    for kbin in range(0, 12):
        f = kbin / (N * dxh)                     # frequency of this bin
        obj = np.exp(2j * np.pi * kbin * xx / N)
        I = orc.forward(d, orc.object_to_spectrum(d, obj))[0]
        if f < fc * 0.999:
            assert np.allclose(I, 1.0, atol=1e-12), kbin
        elif f > fc * 1.001:
            assert np.allclose(I, 0.0, atol=1e-20), kbin


def test_defocus_pupil_properties(orc):
    d0 = tiny(n=32, z=0.0)
    mask, _ = orc.support(d0)
    P0 = orc.pupil_init(d0)
    assert np.allclose(P0[mask], 1.0, atol=0) and np.all(P0[~mask] == 0)
    dp, dm = tiny(n=32, z=12.5), tiny(n=32, z=-12.5)
    Pp, Pm = orc.pupil_init(dp), orc.pupil_init(dm)
    assert np.allclose(np.abs(Pp[mask]), 1.0, atol=1e-14)
    assert np.allclose((Pp * Pm)[mask], 1.0, atol=1e-13)
    # phase against the un-simplified angular-spectrum expression
    n, dk = 32, 1.0 / (32 * dp.pixel_um)
    u, v = np.nonzero(mask)
    k2 = ((u - n // 2) ** 2 + (v - n // 2) ** 2) * dk * dk
    lam = dp.wavelength_um
    phi = 2 * np.pi * 12.5 * (np.sqrt(1 / lam ** 2 - k2) - 1 / lam)
    assert np.allclose(np.angle(Pp[u, v] * np.exp(-1j * phi)), 0.0, atol=1e-9)


# ------------------------------------------------------- offsets and order

def test_offsets_centre_led_and_mirror_symmetry(orc):
    d = tiny(n=64, up=4, grid=15)
    st, off = orc.offsets(d)
    assert st == 0
    assert tuple(off[7 * 15 + 7]) == (0, 0)
    grid = off.reshape(15, 15, 2)
    assert np.array_equal(grid[:, :, 0], -grid[::-1, :, 0])   # drow antisymmetric in r
    assert np.array_equal(grid[:, :, 1], -grid[:, ::-1, 1])   # dcol antisymmetric in c
    assert np.array_equal(grid[:, :, 0], grid[:, :, 1].T)     # square board: x <-> y


def test_offsets_by_trigonometry(orc):
    """Offsets via the illumination angle atan2(d, H) -- an independent route
    to sin(theta) -- round to the same bins (no value within 1e-6 of a tie)."""
    d = tiny(n=64, up=4, grid=15, tile=(312.0, -650.0))
    st, off = orc.offsets(d)
    assert st == 0
    scale = d.n * d.pixel_um / d.wavelength_um
    for r in range(15):
        for c in range(15):
            x = (c - 7) * d.led_pitch_um - d.tile_x_um
            y = (r - 7) * d.led_pitch_um - d.tile_y_um
            rr = math.hypot(x, y)
            th = math.atan2(rr, d.led_height_um)
            sx = math.sin(th) * (x / rr if rr else 0.0)
            sy = math.sin(th) * (y / rr if rr else 0.0)
            for s, got in ((sx, off[r * 15 + c, 1]), (sy, off[r * 15 + c, 0])):
                v = s * scale
                assert abs(v - math.floor(v) - 0.5) > 1e-6
                assert got == math.floor(v + 0.5)


def test_offsets_tile_shift_equals_board_shift(orc):
    """Moving the tile by k LED pitches equals relabelling the LEDs."""
    a = tiny(n=64, up=4, grid=15)
    b = tiny(n=64, up=4, grid=15, tile=(2 * 4000.0, -3 * 4000.0))
    _, oa = orc.offsets(a)
    _, ob = orc.offsets(b)
    ga, gb = oa.reshape(15, 15, 2), ob.reshape(15, 15, 2)
    # LED (r, c) seen from tile b == LED (r + 3, c - 2) seen from tile a
    assert np.array_equal(gb[0:12, 2:15], ga[3:15, 0:13])


def test_offsets_geometry_rejection(orc):
    d = TileDesc(n=64, upsample=3, led_rows=21, led_cols=21)
    st, _ = orc.offsets(d)
    assert st == -2


def test_order_is_increasing_na(orc):
    d = tiny(grid=15)
    o = orc.order(d)
    assert sorted(o.tolist()) == list(range(225))
    r, c = o // 15, o % 15
    key = (2 * r - 14) ** 2 + (2 * c - 14) ** 2
    assert o[0] == 112 and np.all(np.diff(key) >= 0)
    # ties broken by grid index
    for k in range(224):
        if key[k] == key[k + 1]:
            assert o[k] < o[k + 1]


# ------------------------------------------------------------------ groups

def disc_pixels(mask, n, N, off):
    u, v = np.nonzero(mask)
    return set(zip((N // 2 + off[0] - n // 2 + u).tolist(), (N // 2 + off[1] - n // 2 + v).tolist()))


@pytest.mark.parametrize("n,grid,tile", [(16, 5, (0.0, 0.0)), (32, 7, (900.0, 300.0)),
                                         (64, 15, (0.0, 0.0))])
def test_groups_valid_and_first_fit(orc, n, grid, tile):
    d = tiny(n=n, up=4, grid=grid, tile=tile)
    G = orc.groups(d)
    _, off = orc.offsets(d)
    mask, _ = orc.support(d)
    px = [disc_pixels(mask, d.n, d.N, off[j]) for j in range(grid * grid)]
    order = orc.order(d)
    pos = {int(j): k for k, j in enumerate(order)}
    assert sorted(G.sweep.tolist()) == list(range(grid * grid))
    for g in range(G.count):
        mem = G.sweep[G.gstart[g]:G.gstart[g + 1]].tolist()
        assert [pos[j] for j in mem] == sorted(pos[j] for j in mem)     # order kept
        for a in range(len(mem)):
            for b in range(a + 1, len(mem)):
                assert not (px[mem[a]] & px[mem[b]])                    # disjoint
        for j in mem:
            for h in range(g):                                          # first fit
                earlier = G.sweep[G.gstart[h]:G.gstart[h + 1]].tolist()
                assert any(px[j] & px[k] for k in earlier if pos[k] < pos[j])
    if grid == 15 and n == 64:
        assert G.count == 27 and np.diff(G.gstart).max() == 10


# ---------------------------------------------------------- forward model

def test_forward_uniform_object_bright_and_dark_field(orc):
    d = tiny(n=32, up=4, grid=9)
    N = d.N
    I = orc.forward(d, orc.object_to_spectrum(d, np.ones((N, N), complex)))
    _, off = orc.offsets(d)
    r = d.na_obj * d.n * d.pixel_um / d.wavelength_um
    for j in range(81):
        if off[j, 0] ** 2 + off[j, 1] ** 2 <= r * r:
            assert np.allclose(I[j], 1.0, atol=1e-12)
        else:
            assert np.allclose(I[j], 0.0, atol=1e-24)


def test_forward_parseval_and_spectrum_roundtrip(orc):
    td = fpm_synth.TileDraw(desc=tiny(n=16, up=2, grid=5, z=7.0), rng=np.random.default_rng(3))
    obj = fpm_synth.random_object(td.rng, td.desc.N)
    S = orc.object_to_spectrum(td.desc, obj)
    assert rel(orc.spectrum_to_object(td.desc, S), obj) < 1e-13
    # unit object: all energy at the centre bin, n^2
    one = orc.object_to_spectrum(td.desc, np.ones((td.desc.N,) * 2, complex))
    assert abs(one[td.desc.N // 2, td.desc.N // 2] - td.desc.n ** 2) < 1e-9
    P = orc.pupil_init(td.desc)
    I = orc.forward(td.desc, S, P)
    _, off = orc.offsets(td.desc)
    n, N = td.desc.n, td.desc.N
    for j in range(25):
        wy, wx = N // 2 + off[j, 0] - n // 2, N // 2 + off[j, 1] - n // 2
        W = S[wy:wy + n, wx:wx + n]
        assert abs(I[j].sum() - np.sum(abs(P * W) ** 2) / n ** 2) < 1e-10 * max(I[j].sum(), 1)


# -------------------------------------------------------------- the update

def test_fixed_point_true_state_noiseless(orc):
    d = tiny(n=16, up=2, grid=5, z=5.0)
    rng = np.random.default_rng(11)
    obj = fpm_synth.random_object(rng, d.N)
    S = orc.object_to_spectrum(d, obj)
    P = orc.pupil_init(d)
    I = orc.forward(d, S, P).astype(np.float32).astype(np.float64)
    # data exactly representable in float32: recompute S so that it is a
    # fixed point of float32 data is not possible; compare against fp32 noise
    for sched in (0, 1, 2):
        r = orc.reconstruct(d, I, iterations=4, pupil_update=1, schedule=sched, S_in=S, P_in=P)
        assert r.status == 0
        assert rel(r.S, S) < 1e-6 and rel(r.P, P) < 1e-6
        assert np.all(r.residual < 1e-12)


def test_fixed_point_exact_data_fp64(orc):
    """With data that is float32-exact, start the state at the exact solution
    of that data: forward of S_true, then the update must not move."""
    d = tiny(n=16, up=2, grid=3, z=0.0)
    N, n = d.N, d.n
    # object whose LR intensities are exactly 1 (uniform): float32-exact data
    obj = np.ones((N, N), complex)
    S = orc.object_to_spectrum(d, obj)
    P = orc.pupil_init(d)
    I = orc.forward(d, S, P)
    r = orc.reconstruct(d, I.astype(np.float32), iterations=3, pupil_update=1, schedule=0,
                        S_in=S, P_in=P)
    assert rel(r.S, S) < 1e-13 and rel(r.P, P) < 1e-13
    assert np.all(r.residual < 1e-26)


def test_single_led_reduces_to_gerchberg_saxton(orc):
    """One on-axis LED, up = 1, a support covering every bin, pupil off: one
    iteration is a single modulus projection, written with numpy's FFT."""
    n = 16
    d = TileDesc(n=n, upsample=1, led_rows=1, led_cols=1, na_obj=0.8 * 0.532 / 1.625)
    mask, cnt = orc.support(d)
    assert cnt == n * n
    rng = np.random.default_rng(5)
    S0 = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    I = rng.uniform(0.2, 2.0, size=(1, n, n)).astype(np.float32)
    P1 = np.ones((n, n), complex)
    r = orc.reconstruct(d, I, iterations=1, pupil_update=0, schedule=0, S_in=S0, P_in=P1)
    psi = np.fft.ifft2(np.fft.ifftshift(S0))
    psi = np.sqrt(I[0].astype(np.float64)) * psi / np.abs(psi)
    expect = np.fft.fftshift(np.fft.fft2(psi))
    assert rel(r.S, expect) < 1e-12


def test_phase_pupil_update_satisfies_constraint(orc):
    """Spectrum step with a unit-modulus pupil: conj(P) P = 1, so after one
    LED update the new exit spectrum P X' equals the projected spectrum on
    the support (a wrong conjugate or sign breaks this)."""
    d = TileDesc(n=16, upsample=1, led_rows=1, led_cols=1, defocus_um=9.0,
                 na_obj=0.8 * 0.532 / 1.625)
    n = 16
    mask, _ = orc.support(d)
    P = orc.pupil_init(d)
    rng = np.random.default_rng(9)
    S0 = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    I = rng.uniform(0.2, 2.0, size=(1, n, n)).astype(np.float32)
    r = orc.reconstruct(d, I, iterations=1, pupil_update=0, schedule=0, S_in=S0, P_in=P)
    psi = np.fft.ifft2(np.fft.ifftshift(P * S0))
    psi = np.sqrt(I[0].astype(np.float64)) * psi / np.abs(psi)
    proj = np.fft.fftshift(np.fft.fft2(psi))
    assert rel((P * r.S)[mask], proj[mask]) < 1e-12


def test_pupil_recovery_reduces_error_noiseless(orc):
    """Data made with a defocused pupil, reconstruction started from the
    in-focus pupil: with pupil recovery the object error drops below the
    pupil-off error, and the recovered pupil phase moves toward the truth."""
    d = tiny(n=32, up=4, grid=9, z=15.0)
    rng = np.random.default_rng(21)
    obj = fpm_synth.random_object(rng, d.N)
    S = orc.object_to_spectrum(d, obj)
    Ptrue = orc.pupil_init(d)
    I = orc.forward(d, S, Ptrue).astype(np.float32)
    d.defocus_um = 0.0

    def err(res):
        o = orc.spectrum_to_object(d, res.S)
        ph = np.vdot(o, obj)
        return np.linalg.norm(o * ph / abs(ph) - obj) / np.linalg.norm(obj)

    off = orc.reconstruct(d, I, iterations=15, pupil_update=0, schedule=0)
    on = orc.reconstruct(d, I, iterations=15, pupil_update=1, schedule=0)
    assert err(on) < 0.8 * err(off)
    mask, _ = orc.support(d)
    a0 = np.abs(np.vdot(Ptrue[mask], np.ones(mask.sum())))
    a1 = np.abs(np.vdot(Ptrue[mask], on.P[mask] / np.abs(on.P[mask])))
    assert a1 > a0


def test_residual_monotone_noiseless_pupil_off(orc):
    td = fpm_synth.single_tile_64(iterations=8)[0]
    obj, P, I = orc.synthesize(td, noise=False)
    r = orc.reconstruct(td.desc, I, iterations=8, pupil_update=0, schedule=0)
    assert np.all(np.diff(r.residual) <= 1e-12)
    assert r.residual[-1] < 1e-6


def test_grouped_equals_sequential_group_order_bitwise(orc):
    """Sec. 3.2: members of a group touch disjoint spectrum regions, so
    running them from the group-start state equals running them one by one
    in group order -- exactly, with the pupil fixed."""
    d = tiny(n=32, up=4, grid=9, z=4.0)
    rng = np.random.default_rng(4)
    obj = fpm_synth.random_object(rng, d.N)
    I = orc.forward(d, orc.object_to_spectrum(d, obj))
    I = fpm_synth.poisson_noise(rng, I, 1e4)
    a = orc.reconstruct(d, I, iterations=3, pupil_update=0, schedule=1)
    b = orc.reconstruct(d, I, iterations=3, pupil_update=0, schedule=2)
    assert np.array_equal(a.S, b.S) and np.array_equal(a.residual, b.residual)
    c = orc.reconstruct(d, I, iterations=3, pupil_update=0, schedule=0)
    assert not np.array_equal(a.S, c.S)   # the NA order is a different sweep


def test_gauge_invariance_of_forward(orc):
    d = tiny(n=16, up=2, grid=5, z=3.0)
    rng = np.random.default_rng(8)
    S = orc.object_to_spectrum(d, fpm_synth.random_object(rng, d.N))
    P = orc.pupil_init(d)
    s = 1.7
    assert rel(orc.forward(d, S / s, P * s), orc.forward(d, S, P)) < 1e-13
    r = orc.reconstruct(d, orc.forward(d, S, P), iterations=2, pupil_update=1, schedule=0)
    mask, cnt = orc.support(d)
    assert abs(np.sum(np.abs(r.P[mask]) ** 2) - cnt) < 1e-9 * cnt


@pytest.mark.parametrize("grid,tile,noisy,limit", [(9, (-2500.0, 1500.0), False, 0.08),
                                                    (15, (-1072.5, -487.5), True, 0.1)])
def test_off_axis_tile_converges(orc, grid, tile, noisy, limit):
    """A tile away from the optical axis (its centre LED sees a tilted beam)
    must still converge to the object: the initial spectrum has to sit at
    zero frequency, since an intensity image carries no trace of the
    illumination tilt (placing it at the tilted window leaves the estimate
    shifted in frequency, with errors of 20-60 % here)."""
    d = TileDesc(n=64, upsample=4, led_rows=grid, led_cols=grid, tile_x_um=tile[0],
                 tile_y_um=tile[1])
    _, off = orc.offsets(d)
    assert tuple(off[orc.order(d)[0]]) != (0, 0)      # first LED is off-axis here
    rng = np.random.default_rng(31)
    obj = fpm_synth.random_object(rng, d.N)
    I = orc.forward(d, orc.object_to_spectrum(d, obj))
    I = fpm_synth.poisson_noise(rng, I, 1e4) if noisy else I.astype(np.float32)
    r = orc.reconstruct(d, I, iterations=10, pupil_update=0, schedule=1)
    o = orc.spectrum_to_object(d, r.S)
    ph = np.vdot(o, obj)
    ph /= abs(ph)
    assert np.linalg.norm(o * ph - obj) / np.linalg.norm(obj) < limit
