"""Host-side checks of the C-ABI library (no GPU needed): every declared
symbol is exported, and the plan's integer tables (spectrum offsets, order,
LED groups) equal the FP64 oracle's bit for bit."""
import os
import re
import subprocess

import numpy as np
import pytest

import fpm_synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def fpm():
    import paper_2203_02507_amd as fpm
    return fpm


def declared_functions():
    src = open(os.path.join(ROOT, "include", "fpm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fpm_[a-z_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported(fpm):
    names = declared_functions()
    assert len(names) >= 15
    out = subprocess.check_output(["nm", "-D", "--defined-only", fpm.LIB_PATH]).decode()
    exported = set(re.findall(r"\bT (fpm_\w+)", out))
    assert set(names) <= exported, set(names) - exported
    assert set(fpm.EXPORTS) == set(names)
    for n in names:
        getattr(fpm.lib, n)


def _check_tables(fpm, orc, descs):
    plan = fpm.Plan(descs)
    for t, d in enumerate(descs):
        off, order, gof, sweep = plan.tables(t)
        st, ooff = orc.offsets(d)
        assert st == 0
        assert np.array_equal(off, ooff)
        assert np.array_equal(order, orc.order(d))
        G = orc.groups(d)
        assert np.array_equal(gof, G.group_of)
        assert np.array_equal(sweep, G.sweep)
        info = plan.infos[t]
        assert info.ngroups == G.count
        assert info.max_group == int(np.diff(G.gstart).max())
        assert info.support_count == orc.support(d)[1]
        assert info.min_tie_distance > 1e-9
    return plan


def test_plan_matches_oracle_single_tile(fpm, orc):
    d = fpm_synth.single_tile_64()[0].desc
    plan = _check_tables(fpm, orc, [d])
    assert plan.infos[0].ngroups == 27 and plan.infos[0].support_count == 1201
    assert plan.infos[0].steps == 225            # sequential: one LED per step


def test_plan_matches_oracle_full_field(fpm, orc):
    descs = [td.desc for td in fpm_synth.full_fov_tiles()]
    for d in descs[::5]:
        d.defocus_um = 7.5
    plan = _check_tables(fpm, orc, descs[::3])
    assert all(i.steps == i.ngroups for i in plan.infos)   # grouped schedule
    tie = min(fpm.Plan(descs).tile_info(t).min_tie_distance for t in range(256))
    assert 1e-9 < tie < 1e-4          # the full field has a value close to a .5 tie


def test_plan_matches_oracle_uneven(fpm, orc):
    descs = []
    for td in fpm_synth.uneven_batch(T=64):
        if td.desc.n == 256:
            continue
        for up in td.up_candidates:
            td.desc.upsample = up
            if orc.offsets(td.desc)[0] == 0:
                break
        else:
            continue
        descs.append(td.desc)
    assert len(descs) > 20
    _check_tables(fpm, orc, descs)


def test_plan_errors(fpm):
    d = fpm_synth.TileDesc(n=64, upsample=3, led_rows=21, led_cols=21)
    with pytest.raises(fpm.FpmError) as e:
        fpm.Plan([d])
    assert e.value.status == fpm.FPM_E_GEOMETRY
    bad = fpm_synth.TileDesc(n=64, upsample=4, wavelength_um=-1.0)
    with pytest.raises(fpm.FpmError) as e:
        fpm.Plan([bad])
    assert e.value.status == fpm.FPM_E_ARG
    odd = fpm_synth.TileDesc(n=60, upsample=4)
    with pytest.raises(fpm.FpmError) as e:
        fpm.Plan([odd])
    assert e.value.status == fpm.FPM_E_UNSUPPORTED
    nyq = fpm_synth.TileDesc(n=64, upsample=4, na_obj=0.2)
    with pytest.raises(fpm.FpmError) as e:
        fpm.Plan([nyq])
    assert e.value.status == fpm.FPM_E_ARG
    with pytest.raises(fpm.FpmError):
        fpm.Plan([])


def test_host_mode_rejects_bad_intensities_without_gpu_work(fpm):
    """Validation happens on the host before any device call."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("covered by the GPU tests")
    # without a GPU the call must fail cleanly (device or argument error), never crash
    d = fpm_synth.single_tile_64(iterations=1)[0].desc
    plan = fpm.Plan([d])
    I = np.ones((225, 64, 64), np.float32)
    I[3, 2, 1] = np.nan
    with pytest.raises(fpm.FpmError):
        fpm.fpm_reconstruct(plan, I, fpm.FPM_MEM_HOST)


def test_server_without_gpu_fails_cleanly(fpm):
    import torch
    if torch.cuda.is_available():
        pytest.skip("covered by the GPU tests")
    with pytest.raises(fpm.FpmError):
        fpm.Server(1 << 30, 4)
    with pytest.raises(fpm.FpmError) as e:
        fpm.Server(0, 4)
    assert e.value.status == fpm.FPM_E_ARG


def test_precision_flags_plan_identically(fpm):
    """The precision flag changes only the arithmetic of the transforms: the
    plan tables of an MFMA tile are those of the FP32 tile; an unknown
    precision is rejected."""
    base = fpm_synth.full_fov_tiles(only=[17])[0].desc
    plans = []
    for prec in (0, 1, 2):
        d = fpm_synth.full_fov_tiles(only=[17])[0].desc
        d.precision = prec
        plans.append(fpm.Plan([d]).tables(0))
    for other in plans[1:]:
        for a, b in zip(plans[0], other):
            assert np.array_equal(a, b)
    base.precision = 3
    with pytest.raises(fpm.FpmError) as e:
        fpm.Plan([base])
    assert e.value.status == fpm.FPM_E_ARG


def test_n256_plan_tables_and_precision(fpm, orc):
    """256-px tiles plan like the others (tables bit-exact with the oracle);
    the MFMA variant does not run them."""
    rng = np.random.default_rng(256)
    descs = []
    for k in range(3):
        d = fpm_synth.TileDesc(n=256, upsample=3 + k % 2, led_rows=9 + 4 * k, led_cols=9 + 4 * k,
                               tile_x_um=float(rng.uniform(-1500, 1500)),
                               tile_y_um=float(rng.uniform(-1500, 1500)),
                               defocus_um=float(rng.uniform(-30, 30)))
        if orc.offsets(d)[0] == 0:
            descs.append(d)
    assert descs
    _check_tables(fpm, orc, descs)
    d = fpm_synth.TileDesc(n=256, upsample=3, led_rows=9, led_cols=9, precision=1)
    with pytest.raises(fpm.FpmError) as e:
        fpm.Plan([d])
    assert e.value.status == fpm.FPM_E_UNSUPPORTED


def _brute_levels(orc, d, pupil):
    """Level count of the pipelined sweep from pixel coverage: two LEDs
    conflict when some high-resolution pixel lies in both support windows."""
    mask, _ = orc.support(d)
    st, off = orc.offsets(d)
    assert st == 0
    n, N, L = d.n, d.N, d.led_rows * d.led_cols
    uu, vv = np.nonzero(mask)
    cover = {}
    for j in range(L):
        r0 = N // 2 + off[j, 0] - n // 2
        c0 = N // 2 + off[j, 1] - n // 2
        for p in ((r0 + uu) * N + (c0 + vv)).tolist():
            cover.setdefault(p, []).append(j)
    conf = [set([j]) for j in range(L)]
    for leds in cover.values():
        for a in leds:
            conf[a].update(leds)
    last = [0] * L
    top = 0
    for _ in range(d.iterations):
        for j in orc.order(d):
            lv = top + 1 if pupil else 1 + max(last[c] for c in conf[j])
            last[j] = lv
            top = max(top, lv)
    return top


def test_pipelined_levels_match_pixel_coverage(fpm, orc):
    """Sec. 3.2 Fig. 6b/d: the level count of the pipelined sweep equals an
    independent count from pixel coverage; with pupil recovery the levels are
    the sequence; iteration-aligned schedules have iterations x steps levels."""
    d = fpm_synth.single_tile_64(iterations=10, pupil_update=0)[0].desc
    d.schedule = fpm_synth.SCHED_PIPELINED
    info = fpm.Plan([d]).infos[0]
    assert info.levels == _brute_levels(orc, d, pupil=False) == 474
    assert info.steps == d.led_rows * d.led_cols
    d.pupil_update = 1
    assert fpm.Plan([d]).infos[0].levels == 10 * 225
    t = fpm_synth.full_fov_tiles(only=[201], iterations=3, pupil_update=0)[0].desc
    t.schedule = fpm_synth.SCHED_PIPELINED
    assert fpm.Plan([t]).infos[0].levels == _brute_levels(orc, t, pupil=False)
    t.schedule = fpm_synth.SCHED_LED_GROUPS
    i = fpm.Plan([t]).infos[0]
    assert i.levels == 3 * i.steps == 3 * i.ngroups


def test_stitch_rejects_bad_arguments_without_gpu(fpm):
    """Argument checks of fpm_stitch run before any device call."""
    tiles = np.zeros(2 * 2 * 2 * 64 * 64, np.float32)
    out = np.zeros(2 * 128 * 128, np.float32)
    for args in [(2, 2, 64, 40), (0, 2, 64, 8), (2, 2, 64, -1), (2, 2, 1, 0)]:
        with pytest.raises(fpm.FpmError) as e:
            fpm.fpm_stitch(tiles, *args, out, fpm.FPM_MEM_HOST)
        assert e.value.status == fpm.FPM_E_ARG


def test_online_session_state_checks_without_gpu(fpm):
    """The online calls check the session state and the schedule on the host
    before any device call: push / finish without a session -> FPM_E_STATE,
    a non-sequential tile or unequal LED counts -> FPM_E_ARG, abort of no
    session -> OK."""
    d = fpm_synth.single_tile_64(iterations=1)[0].desc
    plan = fpm.Plan([d])
    img = np.ones((64, 64), np.float32)
    with pytest.raises(fpm.FpmError) as e:
        fpm.fpm_online_push(plan, 0, img, fpm.FPM_MEM_HOST)
    assert e.value.status == fpm.FPM_E_STATE
    with pytest.raises(fpm.FpmError) as e:
        fpm.fpm_online_finish(plan, fpm.FPM_MEM_HOST)
    assert e.value.status == fpm.FPM_E_STATE
    assert fpm.fpm_online_abort(plan) == fpm.FPM_OK
    g = fpm_synth.single_tile_64(iterations=1, schedule=fpm_synth.SCHED_LED_GROUPS)[0].desc
    with pytest.raises(fpm.FpmError) as e:
        fpm.fpm_online_begin(fpm.Plan([d, g]))
    assert e.value.status == fpm.FPM_E_ARG
    small = fpm_synth.TileDesc(n=64, upsample=4, led_rows=5, led_cols=5, iterations=1)
    with pytest.raises(fpm.FpmError) as e:
        fpm.fpm_online_begin(fpm.Plan([d, small]))
    assert e.value.status == fpm.FPM_E_ARG
