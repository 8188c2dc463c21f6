"""GPU defocus-distance estimation (Sec. 3.4 Fig. 7b, offline strategy; each
sub-region's own defocus, Sec. 2.2) through the C ABI against the FP64
oracle (oracle/defocus.py) on the same seeded stacks: the candidates'
scores (last-iteration residuals, relative 1e-4 as for every FP32
residual history), the estimate (within 0.05 um of the oracle's, from
scores that agree to that tolerance) and the known z the data were made
with (within 0.5 um); tiles of several sizes and boards in one batched
call, host and device input, and the error cases."""
import dataclasses

import numpy as np
import pytest

import fpm_synth
from oracle import defocus as odf

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fpm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2203_02507_amd as fpm
    return fpm


def cases(orc):
    rng = np.random.default_rng(2203)
    out = []
    for k, (n, rows, up) in enumerate(((64, 15, 4), (128, 15, 4), (96, 13, 3), (64, 21, 4))):
        z = float(rng.uniform(-30.0, 30.0))
        d = fpm_synth.TileDesc(n=n, upsample=up, led_rows=rows, led_cols=rows, iterations=1,
                               defocus_um=z, tile_x_um=float(rng.uniform(-1200, 1200)),
                               tile_y_um=float(rng.uniform(-1200, 1200)))
        _, _, I = orc.synthesize(fpm_synth.TileDraw(desc=d, rng=np.random.default_rng(k)))
        out.append((dataclasses.replace(d, defocus_um=0.0), I, z))
    return out


def test_defocus_estimate_matches_oracle(fpm, orc):
    import torch
    cs = cases(orc)
    descs = [d for d, _, _ in cs]
    I = np.concatenate([x.reshape(-1) for _, x, _ in cs])
    print("tiles: " + ", ".join(f"n={d.n} {d.led_rows}x{d.led_cols}" for d in descs), flush=True)
    z_gpu, s_gpu = fpm.fpm_estimate_defocus(descs, torch.from_numpy(I).cuda(), fpm.FPM_MEM_DEVICE)
    z_host, s_host = fpm.fpm_estimate_defocus(descs, I, fpm.FPM_MEM_HOST)
    assert np.array_equal(z_gpu, z_host) and np.array_equal(s_gpu, s_host)
    for t, (d, It, z_true) in enumerate(cs):
        ref = odf.estimate_defocus(d, It)
        print(f"tile {t}: true {z_true:+.3f} oracle {ref.z_um:+.3f} gpu {z_gpu[t]:+.3f} "
              f"block {ref.block} scores max rel dev "
              f"{float(np.max(np.abs(s_gpu[t] - ref.scores) / ref.scores)):.2e}")
        assert np.allclose(s_gpu[t], ref.scores, rtol=1e-4, atol=0.0), t
        assert int(np.argmin(s_gpu[t])) == ref.best, t
        assert abs(z_gpu[t] - ref.z_um) < 0.05, t
        assert abs(z_gpu[t] - z_true) < 0.5, t


def test_defocus_estimate_errors(fpm):
    d = fpm_synth.TileDesc(n=64, upsample=4, led_rows=15, led_cols=15)
    I = np.ones((225, 64, 64), np.float32)
    with pytest.raises(fpm.FpmError) as e:
        fpm.fpm_estimate_defocus([d], I, fpm.FPM_MEM_HOST, z_step=0.0)
    assert e.value.status == fpm.FPM_E_ARG
    with pytest.raises(fpm.FpmError) as e:
        fpm.fpm_estimate_defocus([d], I, fpm.FPM_MEM_HOST, z_lo=10.0, z_hi=-10.0)
    assert e.value.status == fpm.FPM_E_ARG
    bad = I.copy()
    bad[3, 5, 5] = np.nan
    with pytest.raises(fpm.FpmError) as e:
        fpm.fpm_estimate_defocus([d], bad, fpm.FPM_MEM_HOST)
    assert e.value.status == fpm.FPM_E_ARG
    # a wide pitch leaves the centre LED alone in the aperture
    few = fpm_synth.TileDesc(n=64, upsample=4, led_rows=3, led_cols=3, led_pitch_um=12000.0)
    with pytest.raises(fpm.FpmError) as e:
        fpm.fpm_estimate_defocus([few], np.ones((9, 64, 64), np.float32), fpm.FPM_MEM_HOST)
    assert e.value.status == fpm.FPM_E_GEOMETRY
