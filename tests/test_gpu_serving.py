"""Serving on the GPU: continuous batching must not change any result --
each request is bitwise the same alone and in a mix -- and results match the
FP64 oracle to the FP32 tolerance; admission by device footprint queues
requests that do not fit; cancellation frees a slot without touching others."""
import numpy as np
import pytest

import fpm_synth
from parity import check_windows

pytestmark = pytest.mark.gpu
TOL_OBJ = 1e-4


@pytest.fixture(scope="module")
def fpm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2203_02507_amd as fpm
    return fpm


def requests(orc, count=6, seed=5):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        n = (64, 128)[k % 2]
        grid = (9, 15, 13)[k % 3]
        d = fpm_synth.TileDesc(n=n, upsample=4 if grid > 9 else 3, led_rows=grid, led_cols=grid,
                               iterations=2 + k % 3, schedule=k % 3, pupil_update=(k + 1) % 2,
                               tile_x_um=float(rng.uniform(-1500, 1500)),
                               tile_y_um=float(rng.uniform(-1500, 1500)),
                               defocus_um=float(rng.uniform(-20, 20)))
        td = fpm_synth.TileDraw(desc=d, rng=rng)
        _, _, I = orc.synthesize(td)
        out.append((d, np.ascontiguousarray(I.reshape(-1))))
    return out


def test_alone_equals_mix_and_matches_oracle(fpm, orc):
    reqs = requests(orc)
    srv = fpm.Server(8 << 30, max_slots=16)
    ids = [srv.submit(d, I, fpm.FPM_MEM_HOST) for d, I in reqs]
    mixed = [srv.wait(i, d)[0] for i, (d, _) in zip(ids, reqs)]
    srv.close()
    for k, (d, I) in enumerate(reqs):
        alone_srv = fpm.Server(8 << 30, max_slots=1)
        rid = alone_srv.submit(d, I, fpm.FPM_MEM_HOST)
        alone, stats = alone_srv.wait(rid, d)
        alone_srv.close()
        assert stats.status == fpm.FPM_OK and stats.updates == d.L * d.iterations
        for a, b in zip(alone, mixed[k]):
            assert np.array_equal(a, b), k
        if k < 3:
            r = orc.reconstruct(d, I.reshape(d.L, d.n, d.n))
            o_ref = orc.spectrum_to_object(d, r.S)
            err = np.linalg.norm(alone[0] - o_ref) / np.linalg.norm(o_ref)
            assert err <= TOL_OBJ, (k, err)
            check_windows(orc, d, I.reshape(d.L, d.n, d.n), alone[0], o_ref, 1e-3, f"request {k}")
            assert np.allclose(alone[2], r.residual, rtol=1e-4, atol=1e-9)


def test_served_equals_planned(fpm, orc):
    """A served request and the same tile through fpm_reconstruct agree bitwise."""
    import torch
    d, I = requests(orc, count=2, seed=9)[1]
    srv = fpm.Server(4 << 30, max_slots=4)
    out, _ = srv.wait(srv.submit(d, I, fpm.FPM_MEM_HOST), d)
    srv.close()
    plan = fpm.Plan([d])
    o, p, r = fpm.device_buffers(plan)
    fpm.fpm_reconstruct(plan, torch.from_numpy(I).cuda(), fpm.FPM_MEM_DEVICE, o, p, r)
    torch.cuda.synchronize()
    o = o.cpu().numpy().view(np.complex64).reshape(d.N, d.N)
    assert np.array_equal(o, out[0])


def test_small_budget_queues_and_cancel(fpm, orc):
    """Requests of one shape under a budget that holds one of them: they run
    one after another; a cancelled one reports FPM_E_CANCELLED."""
    rng = np.random.default_rng(17)
    reqs = []
    for k in range(4):
        d = fpm_synth.TileDesc(n=64, upsample=4, led_rows=9, led_cols=9, iterations=3,
                               schedule=1, pupil_update=1, defocus_um=float(rng.uniform(-9, 9)))
        _, _, I = orc.synthesize(fpm_synth.TileDraw(desc=d, rng=rng))
        reqs.append((d, np.ascontiguousarray(I.reshape(-1))))
    d = reqs[0][0]
    one = 2 * d.N * d.N * 8 + d.L * d.n * d.n * 4 + (1 << 20)   # ~ one request's footprint
    srv = fpm.Server(int(1.25 * one), max_slots=8)
    ids = [srv.submit(d, I, fpm.FPM_MEM_HOST) for d, I in reqs]
    srv.cancel(ids[1])
    stats = []
    for k, (i, (d, _)) in enumerate(zip(ids, reqs)):
        if k == 1:
            with pytest.raises(fpm.FpmError) as e:
                srv.wait(i, d)
            assert e.value.status == fpm.FPM_E_CANCELLED
            assert "request cancelled" in str(e.value)  # the message reaches the caller's thread
            continue
        _, st = srv.wait(i, d)
        stats.append(st)
    srv.close()
    adm = sorted(stats, key=lambda s: s.admit_s)
    for a, b in zip(adm, adm[1:]):
        assert b.admit_s >= a.finish_s - 1e-3


def test_submit_rejects_bad_input(fpm, orc):
    d, I = requests(orc, count=1)[0]
    srv = fpm.Server(4 << 30, max_slots=2)
    bad = I.copy()
    bad[5] = np.nan
    with pytest.raises(fpm.FpmError) as e:
        srv.submit(d, bad, fpm.FPM_MEM_HOST)
    assert e.value.status == fpm.FPM_E_ARG
    tiny = fpm.Server(1 << 20, max_slots=2)
    with pytest.raises(fpm.FpmError) as e:
        tiny.submit(d, I, fpm.FPM_MEM_HOST)
    assert e.value.status == fpm.FPM_E_NOMEM
    srv.close()
    tiny.close()
