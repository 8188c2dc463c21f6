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

Every window, and the dark-field-only region, is held to the tolerance or
to a multiple of what the FP64 reference itself cannot pin down there,
whichever is larger.  Both of those limits come from the oracle and the
reference object alone, never from the result under test:

* Conditioning.  Perturbing every intensity by one single-precision
  rounding (relative 2^-24, seeded) moves the oracle's own result; no
  single-precision computation can follow the FP64 trajectory more closely
  than that, so a region's bound is at least COND_FACTOR times that move.
  It matters for sequential sweeps with the pupil fixed: on a 15 x 15 board
  such a perturbation moves a window whose image holds 131 photons by
  1.3e-2 (the GPU differs there by 9e-3), far windows holding a photon or
  two by 0.1 - 0.5, and the dark-field-only region by 3.3e-3 (GPU: 2.6e-3),
  while with pupil recovery and LED groups the same moves stay below 1e-6.
* Representation.  The result comes back as a complex64 object, and
  rounding even the exact object to complex64 moves a window holding
  1e-11 - 1e-9 of the energy by 1e-4 - 1e-3; the FP32 path's own rounding
  grows the same way, like 1/sqrt(share), at about ten times that floor
  (measured on a 21 x 21 board: floor 1.3e-4, GPU 1.4e-3 on a window holding
  7e-10).  A region's bound is at least ROUND_FACTOR times that floor.

Windows the reference leaves empty (EMPTY_SHARE) are skipped.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


COND_FACTOR = 4.0
ROUND_FACTOR = 20.0
# below this share of the spectrum's energy a window holds only the FP64
# transforms' own rounding (~1e-32 of it): the reference leaves it empty
EMPTY_SHARE = 1e-24

# Window and dark-field bounds of the MFMA precision variant, by precision
# (1: split BF16, three terms; 2: scaled FP16).  Scaled FP16 rounds every
# product operand to 11 significant bits relative to the largest value of its
# update (unit roundoff 2^-11 = 4.9e-4).  A dim far-corner window also takes
# the rounding error of every brighter overlapping window's update, 20
# iterations over; on the full-field tiles this reaches ~2e-2 of the window's
# own norm while the whole object stays within 3e-4.  Its window bound is
# therefore 5e-2; the split-BF16 form (~2^-24 per product) is held to 1e-2.
TOL_WIN_MFMA = {1: 1e-2, 2: 5e-2}


@dataclass
class WindowErrors:
    worst: float          # largest relative L2 error over LED support windows
    worst_led: int        # grid index of that LED
    excess: float         # largest error / bound over the windows (<= 1 passes)
    excess_led: int       # grid index of that LED
    measured: int         # windows the reference does not leave empty
    dark_only: float      # relative L2 error over pixels no bright-field LED covers
    dark_bound: float     # its bound
    dark_energy: float    # share of the reference spectrum's energy in that region
    whole: float          # relative L2 error of the whole spectrum

    def __str__(self):
        return (f"window max {self.worst:.2e} (LED {self.worst_led}, {self.measured} windows; "
                f"largest error/bound {self.excess:.2f} at LED {self.excess_led}), dark-only "
                f"{self.dark_only:.2e} (bound {self.dark_bound:.1e}, energy share "
                f"{self.dark_energy:.1e}), whole {self.whole:.2e}")


def _rel(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))


def perturbed_reference(orc, desc, I):
    """The oracle's object from the stack with every intensity moved by one
    single-precision rounding (relative 2^-24, fixed seed)."""
    I = np.asarray(I, dtype=np.float32).reshape(desc.L, desc.n, desc.n)
    xi = np.random.default_rng(24).uniform(-1.0, 1.0, I.shape)
    Ip = (I.astype(np.float64) * (1.0 + 2.0 ** -24 * xi)).astype(np.float32)
    # the pipelined schedule is the sequential sweep (bitwise)
    r = orc.reconstruct(desc, Ip, schedule=0 if desc.schedule == 3 else None)
    assert r.status == 0
    return orc.spectrum_to_object(desc, r.S)


def window_errors(orc, desc, I, o, o_ref, tol) -> WindowErrors:
    """Per-LED-window and dark-field-only errors of object `o` against the
    reference object `o_ref` (both complex [N][N]) and their bounds (tol,
    raised where the reference is ill conditioned or unrepresentable); I is
    the intensity stack [L][n][n] both were reconstructed from."""
    S = orc.object_to_spectrum(desc, np.asarray(o, dtype=np.complex128))
    S_ref = orc.object_to_spectrum(desc, np.asarray(o_ref, dtype=np.complex128))
    # the reference object rounded to the output's complex64
    S_r32 = orc.object_to_spectrum(
        desc, np.asarray(o_ref, dtype=np.complex128).astype(np.complex64).astype(np.complex128))
    # the reference's own response to one single-precision rounding of the data
    S_pert = orc.object_to_spectrum(desc, perturbed_reference(orc, desc, I))
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

    def bound(sel_ref, sel_r32, sel_pert):
        return max(tol, COND_FACTOR * _rel(sel_pert, sel_ref),
                   ROUND_FACTOR * _rel(sel_r32, sel_ref))

    worst, worst_led, excess, excess_led, measured = 0.0, -1, 0.0, -1, 0
    for j in range(desc.L):
        wy = N // 2 + int(off[j][0]) - n // 2
        wx = N // 2 + int(off[j][1]) - n // 2
        sl = (slice(wy, wy + n), slice(wx, wx + n))
        ref_w = S_ref[sl][mask]
        if tot > 0 and float(np.sum(np.abs(ref_w) ** 2)) > EMPTY_SHARE * tot:
            measured += 1
            e = _rel(S[sl][mask], ref_w)
            b = bound(ref_w, S_r32[sl][mask], S_pert[sl][mask])
            if e > worst:
                worst, worst_led = e, j
            if e / b > excess:
                excess, excess_led = e / b, j
        any_cover[sl] |= mask
        if int(off[j][0]) ** 2 + int(off[j][1]) ** 2 <= r2:
            bright_cover[sl] |= mask
    dark = any_cover & ~bright_cover
    share = float(np.sum(np.abs(S_ref[dark]) ** 2)) / tot if tot > 0 else 0.0
    have_dark = dark.any() and float(np.sum(np.abs(S_ref[dark]) ** 2)) > 0
    return WindowErrors(worst=worst, worst_led=worst_led, excess=excess, excess_led=excess_led,
                        measured=measured,
                        dark_only=_rel(S[dark], S_ref[dark]) if have_dark else 0.0,
                        dark_bound=bound(S_ref[dark], S_r32[dark], S_pert[dark])
                        if have_dark else tol,
                        dark_energy=share, whole=_rel(S, S_ref))


def check_windows(orc, desc, I, o, o_ref, tol_window, label=""):
    """Assert the per-window and dark-field-only bounds; return the errors."""
    w = window_errors(orc, desc, I, o, o_ref, tol_window)
    print(f"{label} {w}")
    assert w.excess <= 1.0, (label, str(w))
    assert w.dark_only <= w.dark_bound, (label, str(w))
    return w
