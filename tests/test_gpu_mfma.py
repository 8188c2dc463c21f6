"""GPU parity of the MFMA precision variant: the per-(tile, LED) transforms as
dense centred-DFT products on the matrix cores, in split BF16 (three terms)
and scaled FP16, FP32 accumulation.  Against the FP64 oracle on the same
seeded inputs; tolerance 1e-3 relative L2 on the recovered complex object.
"""
import numpy as np
import pytest

import fpm_synth
from parity import TOL_WIN_MFMA, check_windows

pytestmark = pytest.mark.gpu

TOL_MFMA = 1e-3
TOL_FP32 = 1e-4
TOL_WIN_FP32 = 1e-3
PRECS = [fpm_synth.PREC_MFMA_BF16X3, fpm_synth.PREC_MFMA_FP16]
# Residual histories: residual = sum(|psi| - sqrt I)^2 / sum I, and near
# convergence |psi| - sqrt I is ~3 % of sqrt I, so a relative error eps in
# |psi| moves the residual by ~2 eps / 0.03.  FP16 products carry eps ~ 3e-4
# (-> ~2 %, bound 5 %); split BF16 ~1e-5 (bound 1 %).
RES_RTOL = {fpm_synth.PREC_MFMA_BF16X3: 1e-2, fpm_synth.PREC_MFMA_FP16: 5e-2}


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def fpm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2203_02507_amd as fpm
    return fpm


def run_gpu(fpm, descs, I_list):
    import torch
    plan = fpm.Plan(descs)
    I = torch.from_numpy(np.concatenate([x.reshape(-1) for x in I_list])).cuda()
    obj, pup, res = fpm.device_buffers(plan)
    fpm.fpm_reconstruct(plan, I, fpm.FPM_MEM_DEVICE, obj, pup, res)
    torch.cuda.synchronize()
    return fpm.split_tiles(plan, obj.cpu().numpy(), pup.cpu().numpy(), res.cpu().numpy())


def oracle_run(orc, d, I):
    r = orc.reconstruct(d, I)
    assert r.status == 0
    return orc.spectrum_to_object(d, r.S), r.P, r.residual


@pytest.mark.parametrize("prec", PRECS)
def test_single_tile_mfma_matches_oracle(fpm, orc, prec):
    """64-px tile, 15x15 LEDs, 10 iterations, pupil recovery."""
    td = fpm_synth.single_tile_64()[0]
    _, _, I = orc.synthesize(td)
    o_ref, P_ref, r_ref = oracle_run(orc, td.desc, I)
    td.desc.precision = prec
    o, P, r = run_gpu(fpm, [td.desc], [I])[0]
    err = rel(o, o_ref)
    print(f"precision {prec}: single-tile rel L2 object error vs oracle {err:.3e}, "
          f"pupil {rel(P, P_ref):.3e}")
    assert err <= TOL_MFMA
    assert rel(P, P_ref) <= TOL_MFMA
    check_windows(orc, td.desc, I, o, o_ref, TOL_WIN_MFMA[prec], f"precision {prec}")
    print(f"precision {prec}: residual history max rel dev "
          f"{float(np.max(np.abs(r - r_ref) / np.abs(r_ref))):.2e}")
    assert np.allclose(r, r_ref, rtol=RES_RTOL[prec], atol=1e-9)


@pytest.mark.parametrize("prec", PRECS)
def test_full_field_tiles_mfma_match_oracle(fpm, orc, prec):
    """Four 128-px tiles of the full field (own angles and defocus), LED
    groups with pupil recovery, three iterations; every tile within 1e-3."""
    tds = fpm_synth.full_fov_tiles(only=[0, 37, 120, 255], iterations=3, schedule=1,
                                   pupil_update=1)
    descs, Is = [], []
    for td in tds:
        _, _, I = orc.synthesize(td, z_range=20.0)
        descs.append(td.desc)
        Is.append(I)
    refs = [oracle_run(orc, d, I) for d, I in zip(descs, Is)]
    for d in descs:
        d.precision = prec
    out = run_gpu(fpm, descs, Is)
    errs = [rel(o, ref[0]) for (o, _, _), ref in zip(out, refs)]
    print(f"precision {prec}: per-tile rel L2", " ".join(f"{e:.3e}" for e in errs))
    for t, ((o, P, r), (o_ref, P_ref, r_ref)) in enumerate(zip(out, refs)):
        assert errs[t] <= TOL_MFMA, t
        assert rel(P, P_ref) <= TOL_MFMA, t
        check_windows(orc, descs[t], Is[t], o, o_ref, TOL_WIN_MFMA[prec], f"precision {prec} tile {t}")
        print(f"precision {prec} tile {t}: residual history max rel dev "
              f"{float(np.max(np.abs(r - r_ref) / np.abs(r_ref))):.2e}")
        assert np.allclose(r, r_ref, rtol=RES_RTOL[prec], atol=1e-9), t


def test_mixed_precisions_and_sizes_in_one_plan(fpm, orc):
    """One plan with FP32, BF16x3 and FP16 tiles of 64, 96 and 128 px, each
    schedule: every tile meets its own tolerance, and the FP32 tile is bitwise
    the tile run alone (launch classes do not interact)."""
    rng = np.random.default_rng(2203)
    specs = [(64, 0, 1, 1), (96, 1, 0, 1), (128, 2, 2, 0), (96, 2, 1, 1), (64, 1, 1, 0),
             (128, 1, 0, 1)]
    descs, Is = [], []
    for n, prec, sched, pup in specs:
        d = fpm_synth.TileDesc(n=n, upsample=3 if n == 128 else 4, led_rows=9, led_cols=9,
                               iterations=2, schedule=sched, pupil_update=pup, precision=prec,
                               tile_x_um=float(rng.uniform(-1200, 1200)),
                               tile_y_um=float(rng.uniform(-1200, 1200)),
                               defocus_um=float(rng.uniform(-15, 15)))
        _, _, I = orc.synthesize(fpm_synth.TileDraw(desc=d, rng=rng))
        descs.append(d)
        Is.append(I)
    out = run_gpu(fpm, descs, Is)
    for t, d in enumerate(descs):
        o_ref, _, r_ref = oracle_run(orc, d, Is[t])
        err = rel(out[t][0], o_ref)
        print(f"tile {t} n {d.n} precision {d.precision}: rel L2 {err:.3e}")
        assert err <= (TOL_FP32 if d.precision == 0 else TOL_MFMA), t
        check_windows(orc, d, Is[t], out[t][0], o_ref,
                      TOL_WIN_FP32 if d.precision == 0 else TOL_WIN_MFMA[d.precision],
                      f"tile {t} precision {d.precision}")
    alone = run_gpu(fpm, [descs[0]], [Is[0]])[0]
    assert all(np.array_equal(a, b) for a, b in zip(alone, out[0]))


def test_mfma_edge_cases(fpm, orc):
    """Empty windows (far LEDs of a 21x21 board), a dark stack and a one-LED
    board through the MFMA kernel: finite and within tolerance."""
    d = fpm_synth.TileDesc(n=64, upsample=4, led_rows=21, led_cols=21, iterations=2,
                           schedule=1, pupil_update=1, defocus_um=-7.6,
                           precision=fpm_synth.PREC_MFMA_BF16X3)
    td = fpm_synth.TileDraw(desc=d, rng=np.random.default_rng(3))
    _, _, I = orc.synthesize(td)
    one = fpm_synth.TileDesc(n=96, upsample=2, led_rows=1, led_cols=1, iterations=3,
                             precision=fpm_synth.PREC_MFMA_FP16)
    _, _, I1 = orc.synthesize(fpm_synth.TileDraw(desc=one, rng=np.random.default_rng(4)))
    dark = fpm_synth.TileDesc(n=128, upsample=2, led_rows=3, led_cols=3, iterations=2,
                              precision=fpm_synth.PREC_MFMA_FP16)
    I2 = np.zeros((9, 128, 128), np.float32)
    out = run_gpu(fpm, [d, one, dark], [I, I1, I2])
    for t, (dd, II) in enumerate([(d, I), (one, I1), (dark, I2)]):
        o, P, r = out[t]
        assert np.all(np.isfinite(o)) and np.all(np.isfinite(r)), t
        o_ref, _, r_ref = oracle_run(orc, dd, II)
        if np.linalg.norm(o_ref) == 0:
            assert np.all(o == 0), t
        else:
            assert rel(o, o_ref) <= TOL_MFMA, t
            check_windows(orc, dd, II, o, o_ref, TOL_WIN_MFMA[dd.precision], f"edge case {t}")
