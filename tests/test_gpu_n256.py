"""GPU parity of 256-px tiles (the persistent update kernel whose transposes
go through per-workgroup global scratch) against the FP64 oracle, alone,
mixed with smaller tiles in one plan, through the forward model and through
the server."""
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


def tile256(seed, **kw):
    rng = np.random.default_rng(seed)
    args = dict(n=256, upsample=3, led_rows=9, led_cols=9, iterations=2, schedule=1,
                pupil_update=1, tile_x_um=float(rng.uniform(-1000, 1000)),
                tile_y_um=float(rng.uniform(-1000, 1000)), defocus_um=float(rng.uniform(-30, 30)))
    args.update(kw)
    return fpm_synth.TileDraw(desc=fpm_synth.TileDesc(**args), rng=rng)


def test_forward_n256_matches_oracle(fpm, orc):
    import torch
    td = tile256(11)
    obj = fpm_synth.random_object(td.rng, td.desc.N)
    plan = fpm.Plan([td.desc])
    o = torch.from_numpy(obj.astype(np.complex64).reshape(-1).view(np.float32)).cuda()
    I = torch.empty(plan.total_intensity, dtype=torch.float32, device="cuda")
    fpm.fpm_forward(plan, o, None, I, fpm.FPM_MEM_DEVICE)
    torch.cuda.synchronize()
    got = I.cpu().numpy().reshape(td.desc.L, 256, 256)
    ref = orc.forward(td.desc, orc.object_to_spectrum(td.desc, obj))
    assert rel(got, ref) < 1e-5


@pytest.mark.parametrize("schedule,pupil", [(1, 1), (0, 1), (2, 0)])
def test_n256_tile_matches_oracle(fpm, orc, schedule, pupil):
    td = tile256(20 + schedule, schedule=schedule, pupil_update=pupil)
    _, _, I = orc.synthesize(td)
    o_ref, P_ref, r_ref = oracle_run(orc, td.desc, I)
    o, P, r = run_gpu(fpm, [td.desc], [I])[0]
    err = rel(o, o_ref)
    print(f"n=256 schedule {schedule} pupil {pupil}: rel L2 {err:.3e}")
    assert err <= TOL_OBJ
    assert rel(P, P_ref) <= TOL_OBJ
    check_windows(orc, td.desc, I, o, o_ref, TOL_WIN, f"n=256 schedule {schedule}")
    assert np.allclose(r, r_ref, rtol=1e-4, atol=1e-9)


def test_n256_mixed_with_smaller_tiles(fpm, orc):
    """Two 256-px tiles (more items than one launch's resident workgroups
    would need for a single tile) beside 64- and 128-px tiles in one plan."""
    tds = [tile256(31, led_rows=13, led_cols=13, upsample=4), tile256(32),
           fpm_synth.TileDraw(desc=fpm_synth.TileDesc(n=64, upsample=4, led_rows=9, led_cols=9,
                                                      iterations=2, schedule=1, pupil_update=1),
                              rng=np.random.default_rng(33)),
           fpm_synth.TileDraw(desc=fpm_synth.TileDesc(n=128, upsample=3, led_rows=9, led_cols=9,
                                                      iterations=2, schedule=0, pupil_update=0,
                                                      defocus_um=8.0),
                              rng=np.random.default_rng(34))]
    descs, Is = [], []
    for td in tds:
        _, _, I = orc.synthesize(td)
        descs.append(td.desc)
        Is.append(I)
    out = run_gpu(fpm, descs, Is)
    for t, d in enumerate(descs):
        o_ref, _, r_ref = oracle_run(orc, d, Is[t])
        err = rel(out[t][0], o_ref)
        print(f"tile {t} n {d.n}: rel L2 {err:.3e}")
        assert err <= TOL_OBJ, t
        check_windows(orc, d, Is[t], out[t][0], o_ref, TOL_WIN, f"tile {t}")
        assert np.allclose(out[t][2], r_ref, rtol=1e-4, atol=1e-9), t


def test_n256_served_equals_planned(fpm, orc):
    import torch
    td = tile256(41)
    _, _, I = orc.synthesize(td)
    I = np.ascontiguousarray(I.reshape(-1))
    srv = fpm.Server(4 << 30, max_slots=4)
    out, st = srv.wait(srv.submit(td.desc, I, fpm.FPM_MEM_HOST), td.desc)
    srv.close()
    assert st.status == fpm.FPM_OK
    _, ref = None, run_gpu(fpm, [td.desc], [I])[0]
    assert np.array_equal(out[0], ref[0])


def test_n256_fused_form_bitwise(fpm, orc, monkeypatch):
    """The 256-px kernel with fused cross-lane steps and support pruning
    (the default) gives the bits of the unfused 16-lane form (variant 2) on
    every schedule and pupil mode, and matches the oracle."""
    tds = [tile256(41, schedule=1, pupil_update=1), tile256(42, schedule=0, pupil_update=1),
           tile256(43, schedule=2, pupil_update=0, led_rows=13, led_cols=13)]
    descs, Is = [], []
    for td in tds:
        _, _, I = orc.synthesize(td)
        descs.append(td.desc)
        Is.append(I)
    outs = {}
    for v in ("2", "7"):
        monkeypatch.setenv("FPM_UPDATE_VARIANT_256", v)
        print(f"variant {v}", flush=True)
        outs[v] = run_gpu(fpm, descs, Is)
    for a, b in zip(outs["2"], outs["7"]):
        assert all(np.array_equal(x, y) for x, y in zip(a, b))
    for t, d in enumerate(descs):
        o_ref, _, r_ref = oracle_run(orc, d, Is[t])
        assert rel(outs["7"][t][0], o_ref) <= TOL_OBJ, t
        assert np.allclose(outs["7"][t][2], r_ref, rtol=1e-4, atol=1e-9), t


def test_n256_wide_support_bitwise(fpm, orc, monkeypatch):
    """A support wider than the LDS half holds (NA 0.13: 203 support
    columns > 157) runs the fused form with both transposes in the global
    slot and a smaller pruning; its bits are still those of the unfused
    16-lane form, and it matches the oracle.  Mixed in one launch with an
    NA 0.1 tile, whose launch then takes the same wide path."""
    tds = [tile256(51, na_obj=0.13, upsample=4, schedule=1, pupil_update=1),
           tile256(52, schedule=0, pupil_update=1)]
    descs, Is = [], []
    for td in tds:
        _, _, I = orc.synthesize(td)
        descs.append(td.desc)
        Is.append(I)
    outs = {}
    for v in ("2", "7"):
        monkeypatch.setenv("FPM_UPDATE_VARIANT_256", v)
        print(f"variant {v}", flush=True)
        outs[v] = run_gpu(fpm, descs, Is)
    for a, b in zip(outs["2"], outs["7"]):
        assert all(np.array_equal(x, y) for x, y in zip(a, b))
    o_ref, _, r_ref = oracle_run(orc, descs[0], Is[0])
    err = rel(outs["7"][0][0], o_ref)
    print(f"NA 0.13 tile: rel L2 {err:.3e}")
    assert err <= TOL_OBJ
    assert np.allclose(outs["7"][0][2], r_ref, rtol=1e-4, atol=1e-9)
