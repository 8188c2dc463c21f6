"""Pins for the oracle's online strategy (Sec. 3.4, Fig. 7a): the images arrive
one LED at a time, the first arrival gives the initial guess and the first
iteration updates in arrival order; the later iterations sweep the complete
stack in ascending-NA order.  Each pin ties the online routine to something
fixed outside it: the offline sweep it must reduce to, numpy's FFT for the
initial guess, the split of the run at the first iteration, and the
commutation of updates whose spectrum windows do not meet."""
import numpy as np
import pytest

import fpm_synth
from fpm_synth import TileDesc


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def case(seed=7, n=32, up=4, grid=9, z=0.0, iterations=3):
    d = TileDesc(n=n, upsample=up, led_rows=grid, led_cols=grid, iterations=iterations,
                 defocus_um=z)
    return d


@pytest.fixture(scope="module")
def stack(orc):
    d = case()
    td = fpm_synth.TileDraw(desc=d, rng=np.random.default_rng(31))
    _, _, I = orc.synthesize(td)
    return d, I


@pytest.mark.parametrize("pupil", [0, 1])
def test_online_in_na_order_is_the_offline_sweep(orc, stack, pupil):
    d, I = stack
    a = orc.reconstruct_online(d, I, orc.order(d), pupil_update=pupil)
    b = orc.reconstruct(d, I, pupil_update=pupil, schedule=orc.SEQUENTIAL)
    assert a.status == 0 and b.status == 0
    assert np.array_equal(a.S, b.S) and np.array_equal(a.P, b.P)
    assert np.array_equal(a.residual, b.residual)


def test_initial_guess_is_first_arrival(orc, stack):
    """No iteration: S is zero except the centred n x n window, which holds
    fftshift(fft2(sqrt I_first)) of the first image to arrive."""
    d, I = stack
    rng = np.random.default_rng(4)
    arrival = rng.permutation(d.led_rows * d.led_cols).astype(np.int32)
    r = orc.reconstruct_online(d, I, arrival, iterations=0)
    assert r.status == 0
    n, N = d.n, d.n * d.upsample
    w = np.fft.fftshift(np.fft.fft2(np.sqrt(I[arrival[0]].astype(np.float64))))
    expect = np.zeros((N, N), complex)
    expect[N // 2 - n // 2:N // 2 + n // 2, N // 2 - n // 2:N // 2 + n // 2] = w
    assert rel(r.S, expect) < 1e-13
    assert rel(r.P, orc.pupil_init(d)) == 0.0


def test_split_after_first_iteration(orc, stack):
    """K online iterations = one online iteration, then K-1 offline
    iterations started from its state (the later iterations use the NA order
    and nothing but the state carries over)."""
    d, I = stack
    arrival = np.arange(d.led_rows * d.led_cols, dtype=np.int32)  # raster scan of the board
    full = orc.reconstruct_online(d, I, arrival, iterations=3, pupil_update=1)
    one = orc.reconstruct_online(d, I, arrival, iterations=1, pupil_update=1)
    rest = orc.reconstruct(d, I, iterations=2, pupil_update=1, schedule=orc.SEQUENTIAL,
                           S_in=one.S, P_in=one.P)
    assert np.array_equal(full.S, rest.S) and np.array_equal(full.P, rest.P)
    assert np.array_equal(full.residual, np.concatenate([one.residual, rest.residual]))


def windows(orc, d):
    """Set of spectrum pixels each LED's update touches (its support window)."""
    mask, _ = orc.support(d)
    st, off = orc.offsets(d)
    assert st == 0
    n, N = d.n, d.n * d.upsample
    uu, vv = np.nonzero(mask)
    out = []
    for j in range(d.led_rows * d.led_cols):
        wy, wx = N // 2 + off[j, 0] - n // 2, N // 2 + off[j, 1] - n // 2
        out.append(set(((wy + uu) * N + (wx + vv)).tolist()))
    return out


def test_disjoint_windows_commute_overlapping_do_not(orc, stack):
    """Pupil fixed: two consecutive updates whose support windows in S do not
    meet read and write disjoint pixels, so swapping their arrival leaves S
    bitwise unchanged; swapping two whose windows overlap changes S."""
    d, I = stack
    order = orc.order(d)
    win = windows(orc, d)
    k_dis = next(k for k in range(1, len(order) - 1) if not (win[order[k]] & win[order[k + 1]]))
    k_ovl = next(k for k in range(1, len(order) - 1) if win[order[k]] & win[order[k + 1]])
    base = orc.reconstruct_online(d, I, order, iterations=1, pupil_update=0)

    def swapped(k):
        a = order.copy()
        a[k], a[k + 1] = a[k + 1], a[k]
        return orc.reconstruct_online(d, I, a, iterations=1, pupil_update=0)

    dis = swapped(k_dis)
    assert np.array_equal(dis.S, base.S)
    assert np.allclose(dis.residual, base.residual, rtol=1e-12, atol=0)
    ovl = swapped(k_ovl)
    assert not np.array_equal(ovl.S, base.S)


def test_bad_arrival_rejected(orc, stack):
    d, I = stack
    L = d.led_rows * d.led_cols
    rep = np.arange(L, dtype=np.int32)
    rep[3] = rep[2]
    assert orc.reconstruct_online(d, I, rep).status == -1
    out = np.arange(L, dtype=np.int32)
    out[0] = L
    assert orc.reconstruct_online(d, I, out).status == -1
