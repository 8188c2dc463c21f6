"""GPU parity at the full benchmark size, in the launch configuration the
benchmark times: the 2048-px field cut into 16 x 16 tiles of 128 px (own
angles and defocus), 15 x 15 LEDs, 4x upsampling, 20 iterations, LED groups
with pupil recovery, FP32 path; one captured graph, two chains of tiles, the
autotuned update kernel.

Every tile's intensity stack comes from the FP64 oracle's forward model with
the tile's own shot noise.  Sampled tiles (first, middle, last) are
reconstructed by the oracle one by one and compared element by element
(relative L2 <= 1e-4 on the object and the pupil); all 256 tiles are checked
for properties that hold at any size (finite state, residual falling from
the first to the last iteration), and the sampled tiles of the full batch
are bitwise those of a plan holding only them.  The same batch through the
MFMA DFT path (split BF16 and FP16) matches the same oracle results on the
sampled tiles within 1e-3.  Every sampled result is also bounded on each LED's
support window and on the dark-field-only region of the spectrum (parity.py):
1e-3 for FP32, TOL_WIN_MFMA for the MFMA forms.
"""
from concurrent.futures import ThreadPoolExecutor
import dataclasses
import os

import numpy as np
import pytest

import fpm_synth
from parity import TOL_WIN_MFMA, check_windows

pytestmark = pytest.mark.gpu

TOL = 1e-4
TOL_MFMA = 1e-3
TOL_WIN = 1e-3
SAMPLE = [0, 137, 255]


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def fpm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2203_02507_amd as fpm
    return fpm


def run(fpm, descs, stacks):
    import torch
    plan = fpm.Plan(descs)
    I = torch.from_numpy(np.concatenate([x.reshape(-1) for x in stacks])).cuda()
    obj, pup, res = fpm.device_buffers(plan)
    fpm.fpm_reconstruct(plan, I, fpm.FPM_MEM_DEVICE, obj, pup, res)
    torch.cuda.synchronize()
    return plan, fpm.split_tiles(plan, obj.cpu().numpy(), pup.cpu().numpy(), res.cpu().numpy())


def test_full_field_sampled_tiles_match_oracle(fpm, orc):
    tds = fpm_synth.full_fov_tiles()  # 256 tiles, 20 iterations, LED groups, pupil recovery
    threads = max(1, min(16, os.cpu_count() or 1))
    with ThreadPoolExecutor(threads) as ex:
        stacks = list(ex.map(lambda td: orc.synthesize(td, z_range=20.0)[2], tds))
    descs = [td.desc for td in tds]
    print(f"{len(tds)} oracle-synthesised stacks ready", flush=True)
    plan, out = run(fpm, descs, stacks)
    assert plan.ntiles == 256 and plan.infos[0].N == 512 and plan.infos[0].L == 225

    # properties of every tile
    for t, (o, P, r) in enumerate(out):
        assert np.all(np.isfinite(o)) and np.all(np.isfinite(P)), t
        assert r.shape == (20,) and np.all(np.isfinite(r)), t
        assert r[-1] < r[0], t

    # sampled tiles against the oracle, one tile per thread
    def ref(t):
        r = orc.reconstruct(descs[t], stacks[t])
        assert r.status == 0
        return orc.spectrum_to_object(descs[t], r.S), r.P, r.residual

    with ThreadPoolExecutor(len(SAMPLE)) as ex:
        refs = list(ex.map(ref, SAMPLE))
    for t, (o_ref, P_ref, r_ref) in zip(SAMPLE, refs):
        o, P, r = out[t]
        err, perr = rel(o, o_ref), rel(P, P_ref)
        print(f"tile {t}: rel L2 object {err:.3e} pupil {perr:.3e}", flush=True)
        assert err <= TOL and perr <= TOL, t
        check_windows(orc, descs[t], stacks[t], o, o_ref, TOL_WIN, f"tile {t}")
        assert np.allclose(r, r_ref, rtol=1e-4, atol=1e-9), t

    # the sampled tiles alone: the same bits as in the full batch
    _, alone = run(fpm, [descs[t] for t in SAMPLE], [stacks[t] for t in SAMPLE])
    for k, t in enumerate(SAMPLE):
        assert all(np.array_equal(a, b) for a, b in zip(alone[k], out[t])), t

    # the MFMA DFT path on the same stacks (the oracle's result does not depend on it)
    for prec in (1, 2):
        _, mout = run(fpm, [dataclasses.replace(d, precision=prec) for d in descs], stacks)
        for t, (o_ref, P_ref, _) in zip(SAMPLE, refs):
            err, perr = rel(mout[t][0], o_ref), rel(mout[t][1], P_ref)
            print(f"precision {prec} tile {t}: rel L2 object {err:.3e} pupil {perr:.3e}", flush=True)
            assert err <= TOL_MFMA and perr <= TOL_MFMA, (prec, t)
            check_windows(orc, descs[t], stacks[t], mout[t][0], o_ref, TOL_WIN_MFMA[prec],
                          f"precision {prec} tile {t}")
