"""GPU tests of the chains of tiles: a plan's tiles split into independent
launch sequences on streams of their own (forked from and joined back into
the caller's stream, also under graph capture).  A tile's launches keep their
order, so the result must not depend on the number of chains, nor on graph
replay against eager launches: checked bitwise on a plan that mixes tile
sides (64-256 px, the 256-px kernel with per-chain transpose slots),
schedules (sequential, LED groups, pipelined) and precisions, and against the
FP64 oracle for one tile of each kind.
"""
import numpy as np
import pytest

import fpm_synth
from parity import TOL_WIN_MFMA, check_windows

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def fpm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2203_02507_amd as fpm
    return fpm


def mixed(orc):
    rng = np.random.default_rng(77)
    # (n, schedule, pupil, precision)
    specs = [(256, 1, 1, 0), (128, 1, 1, 0), (64, 0, 1, 0), (96, 3, 0, 0), (256, 0, 0, 0),
             (128, 1, 1, 2), (64, 1, 0, 1), (128, 3, 0, 0), (96, 1, 1, 0)]
    descs, Is = [], []
    for n, sched, pup, prec in specs:
        d = fpm_synth.TileDesc(n=n, upsample=2 if n == 256 else 3, led_rows=7, led_cols=7,
                               iterations=2, schedule=sched, pupil_update=pup, precision=prec,
                               tile_x_um=float(rng.uniform(-800, 800)),
                               tile_y_um=float(rng.uniform(-800, 800)),
                               defocus_um=float(rng.uniform(-10, 10)))
        _, _, I = orc.synthesize(fpm_synth.TileDraw(desc=d, rng=rng))
        descs.append(d)
        Is.append(I)
    return descs, Is


def run(fpm, descs, Is):
    import torch
    plan = fpm.Plan(descs)
    I = torch.from_numpy(np.concatenate([x.reshape(-1) for x in Is])).cuda()
    obj, pup, res = fpm.device_buffers(plan)
    fpm.fpm_reconstruct(plan, I, fpm.FPM_MEM_DEVICE, obj, pup, res)
    fpm.fpm_reconstruct(plan, I, fpm.FPM_MEM_DEVICE, obj, pup, res)  # a replay
    torch.cuda.synchronize()
    return fpm.split_tiles(plan, obj.cpu().numpy(), pup.cpu().numpy(), res.cpu().numpy())


def test_results_do_not_depend_on_chains_or_graph(fpm, orc, monkeypatch):
    descs, Is = mixed(orc)
    outs = {}
    for chains, graph in [(1, True), (2, True), (3, True), (2, False), (4, False)]:
        monkeypatch.setenv("FPM_CHAINS", str(chains))
        if graph:
            monkeypatch.delenv("FPM_NO_GRAPH", raising=False)
        else:
            monkeypatch.setenv("FPM_NO_GRAPH", "1")
        outs[(chains, graph)] = run(fpm, descs, Is)
    ref = outs[(1, True)]
    for key, out in outs.items():
        for t, (a, b) in enumerate(zip(out, ref)):
            assert all(np.array_equal(x, y) for x, y in zip(a, b)), (key, t)
    # one tile of each kind against the oracle
    for t in (0, 2, 3, 5):
        d = descs[t]
        r = orc.reconstruct(d, Is[t], schedule=0 if d.schedule == 3 else d.schedule)
        assert r.status == 0
        o_ref = orc.spectrum_to_object(d, r.S)
        err = rel(ref[t][0], o_ref)
        print(f"tile {t} n {d.n} schedule {d.schedule} precision {d.precision}: rel L2 {err:.3e}")
        assert err <= (1e-4 if d.precision == 0 else 1e-3), t
        check_windows(orc, d, Is[t], ref[t][0], o_ref,
                      1e-3 if d.precision == 0 else TOL_WIN_MFMA[d.precision], f"tile {t}")
