"""GPU parity: the HIP path, called through the C ABI, against the FP64
oracle on the same seeded inputs.

Tolerance: relative L2 error <= 1e-4 on the reconstructed complex object
(FP32 path), as the FP32 target of the method's accuracy budget states; the
integer tables are compared bit for bit in test_plan_cpu.py.  The recovered
spectrum is also bounded on every LED's support window and on the region only
dark-field LEDs reach (relative L2 <= 1e-3 each, see parity.py), which the
whole-object measure cannot see.
"""
import numpy as np
import pytest

import fpm_synth
from parity import check_windows

pytestmark = pytest.mark.gpu

TOL_OBJ = 1e-4
TOL_WIN = 1e-3


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def fpm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2203_02507_amd as fpm
    return fpm


def run_gpu(fpm, descs, I_list, stream=None):
    """Reconstruct on the GPU (device buffers); return per-tile numpy views."""
    import torch
    plan = fpm.Plan(descs)
    I = torch.from_numpy(np.concatenate([x.reshape(-1) for x in I_list])).cuda()
    obj, pup, res = fpm.device_buffers(plan)
    fpm.fpm_reconstruct(plan, I, fpm.FPM_MEM_DEVICE, obj, pup, res)
    torch.cuda.synchronize()
    out = fpm.split_tiles(plan, obj.cpu().numpy(), pup.cpu().numpy(), res.cpu().numpy())
    return plan, out


def oracle_run(orc, d, I):
    r = orc.reconstruct(d, I)
    assert r.status == 0
    return orc.spectrum_to_object(d, r.S), r.P, r.residual


def test_forward_model_matches_oracle(fpm, orc):
    import torch
    tds = fpm_synth.single_tile_64() + fpm_synth.full_fov_tiles(only=[0, 137])
    descs, objs, Ps = [], [], []
    for k, td in enumerate(tds):
        obj = fpm_synth.draw_object_and_defocus(td, None if k == 0 else 20.0)
        descs.append(td.desc)
        objs.append(obj)
    plan = fpm.Plan(descs)
    o = torch.from_numpy(np.concatenate([x.astype(np.complex64).reshape(-1) for x in objs])
                         .view(np.float32)).cuda()
    I = torch.empty(plan.total_intensity, dtype=torch.float32, device="cuda")
    fpm.fpm_forward(plan, o, None, I, fpm.FPM_MEM_DEVICE)
    torch.cuda.synchronize()
    I = I.cpu().numpy()
    for t, (d, obj) in enumerate(zip(descs, objs)):
        info = plan.infos[t]
        got = I[info.intensity_offset:info.intensity_offset + info.L * info.n ** 2]
        got = got.reshape(info.L, info.n, info.n)
        ref = orc.forward(d, orc.object_to_spectrum(d, obj))
        for j in range(info.L):
            scale = max(np.abs(ref[j]).max(), 1e-3 * np.abs(ref).max())
            assert np.abs(got[j] - ref[j]).max() <= 2e-5 * scale + 1e-9, (t, j)
        assert rel(got, ref) < 1e-5


def test_single_tile_sequential_matches_oracle(fpm, orc):
    """64-px tile, 15x15 LEDs, 10 iterations, pupil recovery, NA order."""
    td = fpm_synth.single_tile_64()[0]
    _, _, I = orc.synthesize(td)
    o_ref, P_ref, r_ref = oracle_run(orc, td.desc, I)
    plan, out = run_gpu(fpm, [td.desc], [I])
    o, P, r = out[0]
    err = rel(o, o_ref)
    print("single-tile rel L2 object error vs oracle:", err)
    assert err <= TOL_OBJ
    check_windows(orc, td.desc, I, o, o_ref, TOL_WIN, "single tile")
    assert rel(P, P_ref) <= TOL_OBJ
    assert np.allclose(r, r_ref, rtol=1e-4, atol=1e-9)


@pytest.mark.parametrize("schedule,pupil", [(1, 1), (1, 0), (2, 1), (0, 0)])
def test_multi_tile_schedules_match_oracle(fpm, orc, schedule, pupil):
    """Four 128-px tiles of the full field (own angles and defocus), three
    iterations, each schedule and pupil mode."""
    tds = fpm_synth.full_fov_tiles(only=[0, 37, 120, 255], iterations=3, schedule=schedule,
                                   pupil_update=pupil)
    descs, Is = [], []
    for td in tds:
        _, _, I = orc.synthesize(td, z_range=20.0)
        descs.append(td.desc)
        Is.append(I)
    plan, out = run_gpu(fpm, descs, Is)
    for t, d in enumerate(descs):
        o_ref, P_ref, r_ref = oracle_run(orc, d, Is[t])
        o, P, r = out[t]
        err = rel(o, o_ref)
        print(f"tile {t} schedule {schedule} pupil {pupil}: rel L2 {err:.3e}")
        assert err <= TOL_OBJ
        check_windows(orc, d, Is[t], o, o_ref, TOL_WIN, f"tile {t}")
        assert rel(P, P_ref) <= TOL_OBJ
        assert np.allclose(r, r_ref, rtol=1e-4, atol=1e-9)


def test_grouped_equals_group_order_bitwise_on_gpu(fpm, orc):
    """Pupil fixed: LED groups run concurrently give exactly the result of
    running the same LEDs one at a time in group order (Sec. 3.2)."""
    tds_a = fpm_synth.full_fov_tiles(only=[5, 77], iterations=2, schedule=1, pupil_update=0)
    tds_b = fpm_synth.full_fov_tiles(only=[5, 77], iterations=2, schedule=2, pupil_update=0)
    Is = []
    for td in tds_a:
        obj = fpm_synth.draw_object_and_defocus(td, 20.0)
        S = orc.object_to_spectrum(td.desc, obj)
        Is.append(orc.forward(td.desc, S, orc.pupil_init(td.desc)).astype(np.float32))
    for ta, tb in zip(tds_a, tds_b):
        tb.desc.defocus_um = ta.desc.defocus_um
    _, out_a = run_gpu(fpm, [t.desc for t in tds_a], Is)
    _, out_b = run_gpu(fpm, [t.desc for t in tds_b], Is)
    for (oa, pa, ra), (ob, pb, rb) in zip(out_a, out_b):
        assert np.array_equal(oa, ob)
        assert np.array_equal(pa, pb)


def test_host_and_device_modes_agree(fpm, orc):
    import torch
    td = fpm_synth.single_tile_64(iterations=2)[0]
    _, _, I = orc.synthesize(td)
    plan = fpm.Plan([td.desc])
    N, n = td.desc.N, td.desc.n
    o_h = np.zeros(2 * N * N, np.float32)
    p_h = np.zeros(2 * n * n, np.float32)
    r_h = np.zeros(2, np.float64)
    fpm.fpm_reconstruct(plan, I.reshape(-1).copy(), fpm.FPM_MEM_HOST, o_h, p_h, r_h)
    _, out = run_gpu(fpm, [td.desc], [I])
    assert np.array_equal(o_h.view(np.complex64).reshape(N, N), out[0][0])
    assert np.array_equal(r_h, out[0][2])
    I_bad = I.copy()
    I_bad[7, 3, 3] = -1.0
    with pytest.raises(fpm.FpmError) as e:
        fpm.fpm_reconstruct(plan, I_bad.reshape(-1).copy(), fpm.FPM_MEM_HOST, o_h)
    assert e.value.status == fpm.FPM_E_ARG


def test_mixed_sizes_and_edge_cases(fpm, orc):
    """One plan mixing 64- and 128-px tiles, a one-LED board, zero
    iterations and an all-dark stack."""
    a = fpm_synth.TileDesc(n=64, upsample=3, led_rows=9, led_cols=9, iterations=2,
                           schedule=1, tile_x_um=800.0, tile_y_um=-300.0, defocus_um=-12.0)
    b = fpm_synth.TileDesc(n=128, upsample=2, led_rows=5, led_cols=5, iterations=2,
                           schedule=0, defocus_um=6.0)
    c = fpm_synth.TileDesc(n=64, upsample=2, led_rows=1, led_cols=1, iterations=3)
    z = fpm_synth.TileDesc(n=64, upsample=2, led_rows=3, led_cols=3, iterations=0)
    dark = fpm_synth.TileDesc(n=64, upsample=2, led_rows=3, led_cols=3, iterations=2)
    rng = np.random.default_rng(99)
    descs, Is = [a, b, c, z, dark], []
    for d in descs[:4]:
        td = fpm_synth.TileDraw(desc=d, rng=rng)
        _, _, I = orc.synthesize(td)
        Is.append(I)
    Is.append(np.zeros((9, 64, 64), np.float32))
    _, out = run_gpu(fpm, descs, Is)
    for t, d in enumerate(descs):
        o_ref, P_ref, r_ref = oracle_run(orc, d, Is[t])
        o, P, r = out[t]
        if np.linalg.norm(o_ref) == 0:
            assert np.all(o == 0), t
        else:
            assert rel(o, o_ref) <= TOL_OBJ, t
            check_windows(orc, d, Is[t], o, o_ref, TOL_WIN, f"tile {t}")
        assert np.allclose(r, r_ref, rtol=1e-4, atol=1e-9), t


def test_large_board_far_leds_match_oracle(fpm, orc):
    """21x21 LEDs: the outermost windows are nearly empty at first, so |psi|
    reaches the bottom of the single-precision range; results must stay
    finite and match the oracle."""
    d = fpm_synth.TileDesc(n=64, upsample=4, led_rows=21, led_cols=21, iterations=2,
                           schedule=1, pupil_update=1, defocus_um=-7.6)
    td = fpm_synth.TileDraw(desc=d, rng=np.random.default_rng(3))
    _, _, I = orc.synthesize(td)
    _, out = run_gpu(fpm, [d], [I])
    o, P, r = out[0]
    assert np.all(np.isfinite(o)) and np.all(np.isfinite(r))
    o_ref, P_ref, r_ref = oracle_run(orc, d, I)
    assert rel(o, o_ref) <= TOL_OBJ
    check_windows(orc, d, I, o, o_ref, TOL_WIN, "21x21 board")
    assert np.allclose(r, r_ref, rtol=1e-4, atol=1e-9)


def test_uneven_batch_matches_oracle(fpm, orc):
    """Uneven tiles in one plan: 64/96/128 px, 9x9..21x21 LEDs, upsampling 3-5,
    their own defocus and position; iterations capped at 3 to keep the
    oracle quick.  Every tile compared with the oracle."""
    descs, Is = [], []
    for td in fpm_synth.uneven_batch(T=40, sizes=(64, 96, 128)):
        d = td.desc
        for up in td.up_candidates:
            d.upsample = up
            if orc.offsets(d)[0] == 0:
                break
        else:
            continue
        d.iterations = min(d.iterations, 3)
        _, _, I = orc.synthesize(td)
        descs.append(d)
        Is.append(I)
        if len(descs) == 10:
            break
    assert {d.n for d in descs} == {64, 96, 128}
    _, out = run_gpu(fpm, descs, Is)
    for t, d in enumerate(descs):
        o_ref, P_ref, r_ref = oracle_run(orc, d, Is[t])
        o, P, r = out[t]
        err = rel(o, o_ref)
        print(f"tile {t} n {d.n} grid {d.led_rows} up {d.upsample}: rel L2 {err:.3e}")
        assert err <= TOL_OBJ, t
        check_windows(orc, d, Is[t], o, o_ref, TOL_WIN, f"tile {t}")
        assert np.allclose(r, r_ref, rtol=1e-4, atol=1e-9), t


def _uneven_tiles(indices):
    tds = fpm_synth.uneven_batch(only=indices)
    for td in tds:
        d = td.desc
        for up in td.up_candidates:
            d.upsample = up
            if fpm_synth_offsets_ok(d):
                break
    return tds


def fpm_synth_offsets_ok(d):
    import oracle
    return oracle.offsets(d)[0] == 0


@pytest.mark.timeout(900)
def test_uneven_tiles_at_drawn_iterations_match_oracle(fpm, orc):
    """Tiles of the 512-tile uneven batch at the iteration counts they drew
    (no cap), in one plan: a 256-px tile on a 21x21 board (441 LEDs, 5x
    upsampling, 21 iterations), a 96-px tile on 13x13 LEDs (29 iterations)
    and a 64-px tile on 13x13 LEDs (5x upsampling, 28 iterations).  Far dark-field windows
    of a large board hold ~1e-10 of the energy; late iterations there are
    where single precision runs out first."""
    tds = _uneven_tiles([95, 22, 11])
    got = sorted((td.desc.n, td.desc.led_rows, td.desc.iterations) for td in tds)
    assert got == [(64, 13, 28), (96, 13, 29), (256, 21, 21)], got
    descs, Is = [], []
    for td in tds:
        _, _, I = orc.synthesize(td)
        descs.append(td.desc)
        Is.append(I)
    _, out = run_gpu(fpm, descs, Is)
    for t, d in enumerate(descs):
        o, P, r = out[t]
        assert np.all(np.isfinite(o)) and np.all(np.isfinite(r)), t
        o_ref, P_ref, r_ref = oracle_run(orc, d, Is[t])
        err = rel(o, o_ref)
        print(f"tile n {d.n} grid {d.led_rows} up {d.upsample} iters {d.iterations}: "
              f"rel L2 {err:.3e}, pupil {rel(P, P_ref):.3e}")
        assert err <= TOL_OBJ, t
        assert rel(P, P_ref) <= TOL_OBJ, t
        check_windows(orc, d, Is[t], o, o_ref, TOL_WIN, f"n {d.n}")
        assert np.allclose(r, r_ref, rtol=1e-4, atol=1e-9), t


@pytest.mark.parametrize("n", [64, 96, 128])
def test_update_variants(fpm, orc, monkeypatch, n):
    """The autotuner's variants: 4 or 8 lanes per line, LDS row padding, one
    or several rounds of lines per workgroup (6, 7: 8 lanes in two and four
    rounds, with the fused cross-lane steps; 8: 4 lanes in two rounds).
    Variants of one lane count differ only in layout (and in how the 8-lane
    cross-lane steps are issued) and give the same bits; the 8-lane form
    orders its floating-point steps differently and must meet the same
    tolerance against the oracle."""
    rng = np.random.default_rng(n)
    descs, Is = [], []
    for k in range(2):
        d = fpm_synth.TileDesc(n=n, upsample=3, led_rows=9, led_cols=9, iterations=2, schedule=1,
                               pupil_update=1, tile_x_um=float(rng.uniform(-1000, 1000)),
                               tile_y_um=float(rng.uniform(-1000, 1000)),
                               defocus_um=float(rng.uniform(-20, 20)))
        _, _, I = orc.synthesize(fpm_synth.TileDraw(desc=d, rng=rng))
        descs.append(d)
        Is.append(I)
    refs = [oracle_run(orc, d, I) for d, I in zip(descs, Is)]
    first = {}
    for v in range(9):
        monkeypatch.setenv("FPM_UPDATE_VARIANT", str(v))
        _, out = run_gpu(fpm, descs, Is)
        fam = 4 if v < 4 or v == 8 else 8
        if fam not in first:
            first[fam] = out
            for (o, _, r), (o_ref, _, r_ref) in zip(out, refs):
                assert rel(o, o_ref) <= TOL_OBJ, v
                assert np.allclose(r, r_ref, rtol=1e-4, atol=1e-9), v
        else:
            for a, b in zip(out, first[fam]):
                assert all(np.array_equal(x, y) for x, y in zip(a, b)), v
    for a, b in zip(first[4], first[8]):
        assert rel(a[0], b[0]) < 1e-5


def test_group_sequential_form_bitwise(fpm, orc, monkeypatch):
    """One workgroup per tile group (members in slot order, pupil mean applied
    by the last member) gives the bits of the concurrent form with its
    separate group-mean kernel, for every schedule and pupil mode."""
    tds = fpm_synth.full_fov_tiles(only=[9, 70, 140], iterations=2, schedule=1, pupil_update=1)
    descs, Is = [], []
    for k, td in enumerate(tds):
        _, _, I = orc.synthesize(td, z_range=20.0)
        td.desc.schedule = (1, 0, 2)[k]
        td.desc.pupil_update = (1, 1, 0)[k]
        descs.append(td.desc)
        Is.append(I)
    out = {}
    for seq in ("0", "1"):
        monkeypatch.setenv("FPM_GROUP_SEQ", seq)
        _, out[seq] = run_gpu(fpm, descs, Is)
    diffs = [(t, k, float(np.abs(x - y).max()))
             for t, (a, b) in enumerate(zip(out["0"], out["1"]))
             for k, (x, y) in enumerate(zip(a, b)) if not np.array_equal(x, y)]
    assert not diffs, diffs
    for t, d in enumerate(descs):
        o_ref, _, _ = oracle_run(orc, d, Is[t])
        assert rel(out["1"][t][0], o_ref) <= TOL_OBJ


@pytest.mark.parametrize("pupil", [0, 1])
def test_pipelined_equals_sequential_bitwise(fpm, orc, pupil):
    """Sec. 3.2 Fig. 6b/d: the level-scheduled sweep over all iterations gives
    the bits of the sequential NA-order sweep, in a plan that also holds tiles
    of the other schedules; the sequential result is checked against the
    oracle."""
    tds = fpm_synth.full_fov_tiles(only=[12, 100, 190], iterations=3, schedule=0,
                                   pupil_update=pupil)
    descs, Is = [], []
    for td in tds:
        _, _, I = orc.synthesize(td, z_range=20.0)
        descs.append(td.desc)
        Is.append(I)
    other = fpm_synth.TileDesc(n=64, upsample=4, led_rows=9, led_cols=9, iterations=2,
                               schedule=1, pupil_update=1)
    _, _, I_other = orc.synthesize(fpm_synth.TileDraw(desc=other, rng=np.random.default_rng(8)))
    _, seq = run_gpu(fpm, descs + [other], Is + [I_other])
    import copy
    piped = [copy.copy(d) for d in descs]
    for d in piped:
        d.schedule = fpm_synth.SCHED_PIPELINED
    plan, pip = run_gpu(fpm, piped + [other], Is + [I_other])
    if pupil == 0:
        assert all(i.levels < i.iterations * i.L for i in plan.infos[:3])
    for a, b in zip(seq, pip):
        assert all(np.array_equal(x, y) for x, y in zip(a, b))
    for t, d in enumerate(descs):
        o_ref, _, r_ref = oracle_run(orc, d, Is[t])
        assert rel(pip[t][0], o_ref) <= TOL_OBJ
        check_windows(orc, d, Is[t], pip[t][0], o_ref, TOL_WIN, f"pipelined tile {t}")
        assert np.allclose(pip[t][2], r_ref, rtol=1e-4, atol=1e-9)


def test_device_mode_errors_write_no_output(fpm, orc):
    """Device mode checks its intensities before the sweep and its residuals
    after it; on a failed check no output is written and fpm_plan_status
    reports FPM_E_ARG or FPM_E_DIVERGED; host mode returns the same errors
    with its outputs untouched; a good call afterwards is unaffected."""
    import torch
    td = fpm_synth.single_tile_64(iterations=2)[0]
    _, _, I = orc.synthesize(td)
    plan = fpm.Plan([td.desc])
    nan_I = I.copy()
    nan_I[11, 7, 9] = np.nan
    big_I = I.copy()
    big_I[5, 20, 0] = 3e38   # finite, but two of them in one lane's row segment
    big_I[5, 20, 1] = 3e38   # overflow its FP32 residual partial: inf / inf
    for bad, code in ((nan_I, fpm.FPM_E_ARG), (big_I, fpm.FPM_E_DIVERGED)):
        print(f"device mode, expecting status {code}", flush=True)
        obj = torch.full((plan.total_object * 2,), 7.0, dtype=torch.float32, device="cuda")
        pup = torch.full((plan.total_pupil * 2,), 7.0, dtype=torch.float32, device="cuda")
        res = torch.full((plan.total_residual,), 7.0, dtype=torch.float64, device="cuda")
        fpm.fpm_reconstruct(plan, torch.from_numpy(bad.reshape(-1).copy()).cuda(),
                            fpm.FPM_MEM_DEVICE, obj, pup, res)
        assert fpm.fpm_plan_status(plan) == code
        assert bool(torch.all(obj == 7.0)) and bool(torch.all(pup == 7.0))
        assert bool(torch.all(res == 7.0))
        o_h = np.full(plan.total_object * 2, 7.0, np.float32)
        r_h = np.full(plan.total_residual, 7.0, np.float64)
        with pytest.raises(fpm.FpmError) as e:
            fpm.fpm_reconstruct(plan, bad.reshape(-1).copy(), fpm.FPM_MEM_HOST, o_h, None, r_h)
        assert e.value.status == code
        assert np.all(o_h == 7.0) and np.all(r_h == 7.0)
    plan2, out = run_gpu(fpm, [td.desc], [I])
    o_ref, _, r_ref = oracle_run(orc, td.desc, I)
    assert rel(out[0][0], o_ref) <= TOL_OBJ
    assert fpm.fpm_plan_status(plan2) == fpm.FPM_OK


@pytest.mark.parametrize("na", [0.05, 0.15])
def test_support_widths_bitwise_across_variants(fpm, orc, monkeypatch, na):
    """Narrow and wide supports (NA 0.05 / 0.15: pruning Z = 5 / 0 at n = 128,
    Z = 3 / 0 at n = 96) through the round form's row-segment gather and
    update and its swizzled LDS rows: the four-round variant gives the bits
    of the one-round 8-lane variant, and both match the oracle."""
    rng = np.random.default_rng(int(na * 1000))
    descs, Is = [], []
    for n, up in ((128, 2), (96, 3)):
        d = fpm_synth.TileDesc(n=n, upsample=up, led_rows=7, led_cols=7, iterations=2, schedule=1,
                               pupil_update=1, na_obj=na, tile_x_um=float(rng.uniform(-600, 600)),
                               tile_y_um=float(rng.uniform(-600, 600)),
                               defocus_um=float(rng.uniform(-10, 10)))
        _, _, I = orc.synthesize(fpm_synth.TileDraw(desc=d, rng=rng))
        descs.append(d)
        Is.append(I)
    outs = {}
    for v in ("4", "7"):
        monkeypatch.setenv("FPM_UPDATE_VARIANT", v)
        print(f"NA {na} variant {v}", flush=True)
        _, outs[v] = run_gpu(fpm, descs, Is)
    for a, b in zip(outs["4"], outs["7"]):
        assert all(np.array_equal(x, y) for x, y in zip(a, b))
    for t, d in enumerate(descs):
        o_ref, _, r_ref = oracle_run(orc, d, Is[t])
        o, _, r = outs["7"][t]
        print(f"n {d.n} NA {na}: rel L2 {rel(o, o_ref):.3e}")
        assert rel(o, o_ref) <= TOL_OBJ, t
        check_windows(orc, d, Is[t], o, o_ref, TOL_WIN, f"n {d.n} NA {na}")
        assert np.allclose(r, r_ref, rtol=1e-4, atol=1e-9), t
