"""Error measures shared by the GPU parity tests.

The relative L2 error of the whole object is dominated by the bright-field
part of the spectrum: the pixels that only dark-field LEDs reach (the part of
the spectrum that Fourier ptychography synthesises, Sec. 1 / Sec. 2.1) hold a
few millionths of its energy, so a whole-object bound cannot see errors
there.  These helpers measure the error of the recovered spectrum on each
LED's support window separately and on the dark-field-only region, and the
tests bound those too.

The spectrum of a result is taken from its object with the oracle's FP64
transform (S = shift FFT_N(o) / up^2), so the measure includes the
finalisation step of the path under test.

Windows holding less than SHARE_FLOOR of the reference spectrum's energy are
not bounded one by one: the object comes back in complex64, and rounding an
exact object to complex64 alone already moves such a window by ~1e-3 (the
far corner LEDs of a 15x15 board after a few iterations hold ~1e-11 of the
energy).  Above the floor the same rounding moves a window by <= 5e-5.  The
dark-field-only region is bounded as a whole in every case.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


SHARE_FLOOR = 1e-10

# Window and dark-field bounds of the MFMA precision variant, by precision
# (1: split BF16, three terms; 2: scaled FP16).
TOL_WIN_MFMA = {1: 1e-2, 2: 1e-2}


@dataclass
class WindowErrors:
    worst: float          # largest relative L2 error over LED support windows
    measured: int         # windows above the energy floor (the others: see above)
    worst_led: int        # grid index of that LED
    dark_only: float      # relative L2 error over pixels no bright-field LED covers
    dark_energy: float    # share of the reference spectrum's energy in that region
    whole: float          # relative L2 error of the whole spectrum

    def __str__(self):
        return (f"window max {self.worst:.2e} (LED {self.worst_led}, {self.measured} windows), "
                f"dark-only "
                f"{self.dark_only:.2e} (energy share {self.dark_energy:.1e}), "
                f"whole {self.whole:.2e}")


def _rel(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))


def window_errors(orc, desc, o, o_ref) -> WindowErrors:
    """Per-LED-window and dark-field-only errors of object `o` against the
    reference object `o_ref` (both complex [N][N])."""
    S = orc.object_to_spectrum(desc, np.asarray(o, dtype=np.complex128))
    S_ref = orc.object_to_spectrum(desc, np.asarray(o_ref, dtype=np.complex128))
    mask, _ = orc.support(desc)
    st, off = orc.offsets(desc)
    assert st == 0
    n, N = desc.n, desc.N
    # support radius in bins, as the support mask has it
    c = n // 2
    r2 = max((u - c) ** 2 + (v - c) ** 2 for u, v in zip(*np.nonzero(mask)))
    bright_cover = np.zeros((N, N), bool)
    any_cover = np.zeros((N, N), bool)
    tot = float(np.sum(np.abs(S_ref) ** 2))
    worst, worst_led, measured = 0.0, -1, 0
    for j in range(desc.L):
        wy = N // 2 + int(off[j][0]) - n // 2
        wx = N // 2 + int(off[j][1]) - n // 2
        sl = (slice(wy, wy + n), slice(wx, wx + n))
        ref_w = S_ref[sl][mask]
        if tot > 0 and float(np.sum(np.abs(ref_w) ** 2)) >= SHARE_FLOOR * tot:
            measured += 1
            e = _rel(S[sl][mask], ref_w)
            if e > worst:
                worst, worst_led = e, j
        any_cover[sl] |= mask
        if int(off[j][0]) ** 2 + int(off[j][1]) ** 2 <= r2:
            bright_cover[sl] |= mask
    dark = any_cover & ~bright_cover
    share = float(np.sum(np.abs(S_ref[dark]) ** 2)) / tot if tot > 0 else 0.0
    return WindowErrors(worst=worst, measured=measured, worst_led=worst_led,
                        dark_only=_rel(S[dark], S_ref[dark]) if dark.any() else 0.0,
                        dark_energy=share, whole=_rel(S, S_ref))


def check_windows(orc, desc, o, o_ref, tol_window, label=""):
    """Assert the per-window and dark-field-only bounds; return the errors."""
    w = window_errors(orc, desc, o, o_ref)
    print(f"{label} {w}")
    assert w.worst <= tol_window, (label, str(w))
    assert w.dark_only <= tol_window, (label, str(w))
    return w
