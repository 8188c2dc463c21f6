"""Pins for the parts of the FP64 oracle that the round-trip pins cannot see:
the pupil step of an LED group (the mean of its members' increments, Sec. 3.2
grouping with the embedded pupil update), the residual (the running
amplitude residual sum (|psi| - sqrt I)^2 / sum I), and the normalisation of
the pupil step (the largest squared magnitude over the whole high-resolution
spectrum at the start of the iteration).

Each pin compares the oracle with something it does not compute itself: a
different schedule of the same oracle on a board where the two must agree,
single-LED runs of the same oracle combined by hand, numpy's FFT, or the
scaling of one input.  A plausible slip -- a sum instead of a mean, a
division by the LED count instead of the group size, |psi|^2 - I instead of
|psi| - sqrt I, a per-window instead of a whole-spectrum maximum -- fails at
least one of them."""
import numpy as np
import pytest

from fpm_synth import TileDesc


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def rnd_state(rng, d, scale=1.0):
    N = d.N
    return scale * (rng.normal(size=(N, N)) + 1j * rng.normal(size=(N, N)))


def gauge(S_in, S_out, px):
    """The end-of-iteration pupil normalisation multiplies P by s and divides
    S by s; on a pixel no LED window touches, S_out = S_in / s."""
    return float((S_in[px] / S_out[px]).real)


def test_groups_of_one_equal_sequential_with_pupil(orc):
    """Every LED's support overlaps every other LED's (a 3x3 board with 1 mm
    pitch), so each LED group has one member.  The group mean of one
    increment is the increment itself: with pupil recovery on, the grouped
    sweep equals the sequential one bit for bit (a division by the LED count
    instead of the group size breaks this)."""
    d = TileDesc(n=32, upsample=2, led_rows=3, led_cols=3, led_pitch_um=1000.0,
                 defocus_um=6.0, iterations=3)
    g = orc.groups(d)
    assert g.count == d.L and np.all(np.diff(g.gstart) == 1)
    assert np.array_equal(g.sweep, orc.order(d))
    rng = np.random.default_rng(11)
    I = rng.uniform(0.1, 2.0, size=(d.L, d.n, d.n)).astype(np.float32)
    a = orc.reconstruct(d, I, iterations=3, pupil_update=1, schedule=1)
    b = orc.reconstruct(d, I, iterations=3, pupil_update=1, schedule=0)
    assert np.array_equal(a.S, b.S)
    assert np.array_equal(a.P, b.P)
    assert np.array_equal(a.residual, b.residual)


def _board(cols, x0, pitch=20000.0):
    # n = 32, 3x upsampling: LED windows 20 mm apart at 90 mm height are
    # ~21 bins apart, more than the support diameter (2 r = 19.5 bins)
    return TileDesc(n=32, upsample=3, led_rows=1, led_cols=cols, led_pitch_um=pitch,
                    led_origin_x_um=x0, defocus_um=5.0, iterations=1)


def test_group_pupil_step_is_mean_of_member_increments(orc):
    """A 1x3 board whose three supports are disjoint forms one group of three.
    One grouped iteration from (S_in, P_in) must give the pupil
    P_in + (dP_0 + dP_1 + dP_2) / 3, where dP_j is the increment LED j makes
    alone from the same state (a 1x1 board with that LED); each member's
    spectrum pixels equal its single-LED result.  Summing the increments
    instead of averaging them breaks this."""
    d3 = _board(3, 0.0)
    g = orc.groups(d3)
    assert g.count == 1 and g.gstart[1] - g.gstart[0] == 3
    _, off3 = orc.offsets(d3)
    rng = np.random.default_rng(5)
    S_in = rnd_state(rng, d3)
    P_in = orc.pupil_init(d3)
    I3 = rng.uniform(0.1, 2.0, size=(3, d3.n, d3.n)).astype(np.float32)
    far = (0, 0)   # no LED window of this board reaches the corner pixel
    rg = orc.reconstruct(d3, I3, iterations=1, pupil_update=1, schedule=1, S_in=S_in, P_in=P_in)
    s_g = gauge(S_in, rg.S, far)
    P_pre_g = rg.P / s_g
    S_pre_g = rg.S * s_g
    incs = []
    mask, _ = orc.support(d3)
    N, n = d3.N, d3.n
    for c in range(3):
        d1 = _board(1, (c - 1) * 20000.0)
        _, off1 = orc.offsets(d1)
        assert np.array_equal(off1[0], off3[c])
        r1 = orc.reconstruct(d1, I3[c:c + 1], iterations=1, pupil_update=1, schedule=0,
                             S_in=S_in, P_in=P_in)
        s1 = gauge(S_in, r1.S, far)
        incs.append(r1.P / s1 - P_in)
        # the member's own support pixels of the spectrum
        wy = N // 2 + off3[c][0] - n // 2
        wx = N // 2 + off3[c][1] - n // 2
        win_g = S_pre_g[wy:wy + n, wx:wx + n][mask]
        win_1 = (r1.S * s1)[wy:wy + n, wx:wx + n][mask]
        assert rel(win_g, win_1) < 1e-13
    expect = P_in + (incs[0] + incs[1] + incs[2]) / 3.0
    assert rel(P_pre_g, expect) < 1e-13
    # the increments are not negligible: a sum would be far off
    assert rel(P_in + incs[0] + incs[1] + incs[2], expect) > 1e-2


def test_residual_of_one_update_by_numpy(orc):
    """One LED, pupil fixed, one iteration from (S_in, P_in): the residual is
    sum (|psi| - sqrt I)^2 / sum I with psi the low-resolution field of the
    starting state, evaluated here with numpy's FFT.  The |psi|^2 - I form
    gives a different number."""
    d = TileDesc(n=32, upsample=2, led_rows=1, led_cols=1, led_origin_x_um=3000.0,
                 defocus_um=-7.0, iterations=1)
    rng = np.random.default_rng(17)
    S_in = rnd_state(rng, d, 0.05)
    P_in = orc.pupil_init(d)
    I = rng.uniform(0.0, 3.0, size=(1, d.n, d.n)).astype(np.float32)
    I[0, 3, 4] = 0.0
    r = orc.reconstruct(d, I, iterations=1, pupil_update=0, schedule=0, S_in=S_in, P_in=P_in)
    _, off = orc.offsets(d)
    n, N = d.n, d.N
    wy = N // 2 + off[0][0] - n // 2
    wx = N // 2 + off[0][1] - n // 2
    X = S_in[wy:wy + n, wx:wx + n]
    psi = np.fft.ifft2(np.fft.ifftshift(P_in * X))
    I64 = I[0].astype(np.float64)
    expect = np.sum((np.abs(psi) - np.sqrt(I64)) ** 2) / np.sum(I64)
    assert abs(r.residual[0] - expect) <= 1e-12 * expect
    wrong = np.sum((np.abs(psi) ** 2 - I64) ** 2) / np.sum(I64)
    assert abs(wrong - expect) > 1e-3 * expect


def test_pupil_step_normalised_by_whole_spectrum_maximum(orc):
    """Raising |S| at a pixel outside the LED's window to a new maximum
    leaves the spectrum step unchanged and scales the pupil increment by the
    ratio of the old to the new maximum of |S|^2: the pupil step is divided
    by the largest |S|^2 over the whole spectrum (taken at the start of the
    iteration), not over the LED's window."""
    d = TileDesc(n=32, upsample=2, led_rows=1, led_cols=1, defocus_um=4.0, iterations=1)
    rng = np.random.default_rng(23)
    S_a = rnd_state(rng, d)
    P_in = orc.pupil_init(d)
    I = rng.uniform(0.1, 2.0, size=(1, d.n, d.n)).astype(np.float32)
    big, probe = (1, 2), (0, 0)    # both outside the centred 32x32 window of N = 64
    S_b = S_a.copy()
    m_a = np.max(np.abs(S_a) ** 2)
    S_b[big] = 7.0 * np.sqrt(m_a)
    m_b = np.max(np.abs(S_b) ** 2)
    ra = orc.reconstruct(d, I, iterations=1, pupil_update=1, schedule=0, S_in=S_a, P_in=P_in)
    rb = orc.reconstruct(d, I, iterations=1, pupil_update=1, schedule=0, S_in=S_b, P_in=P_in)
    sa, sb = gauge(S_a, ra.S, probe), gauge(S_b, rb.S, probe)
    dPa = ra.P / sa - P_in
    dPb = rb.P / sb - P_in
    assert rel(dPb, dPa * (m_a / m_b)) < 1e-12
    n, N = d.n, d.N
    w = slice(N // 2 - n // 2, N // 2 + n // 2)
    assert rel((rb.S * sb)[w, w], (ra.S * sa)[w, w]) < 1e-13
    assert m_b / m_a == pytest.approx(49.0)
