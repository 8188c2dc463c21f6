"""GPU stitching (Sec. 3.1, Eq. (1)) through the C ABI against the FP64
oracle: random tiles on several grids, sides and overlaps (tiles that agree
on their overlaps up to unknown global factors, and tiles that do not), host
and device modes, and the stitched field of reconstructed full-field tiles."""
import numpy as np
import pytest

import fpm_synth
from oracle import stitch as ost

pytestmark = pytest.mark.gpu
TOL = 1e-6


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def fpm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2203_02507_amd as fpm
    return fpm


def gpu_stitch(fpm, tiles, overlap):
    import torch
    R, C = len(tiles), len(tiles[0])
    side = tiles[0][0].shape[0]
    arr = np.stack([np.stack(r) for r in tiles]).astype(np.complex64)
    H, W = fpm.stitched_shape(R, C, side, overlap)
    src = torch.from_numpy(arr.reshape(-1).view(np.float32)).cuda()
    out = torch.empty(2 * H * W, dtype=torch.float32, device="cuda")
    fpm.fpm_stitch(src, R, C, side, overlap, out, fpm.FPM_MEM_DEVICE)
    return out.cpu().numpy().view(np.complex64).reshape(H, W)


@pytest.mark.parametrize("grid,side,ov,consistent", [
    ((1, 1), 64, 0, False), ((1, 3), 64, 16, True), ((3, 1), 96, 10, False),
    ((2, 2), 128, 26, True), ((4, 5), 64, 8, False), ((3, 3), 256, 32, True),
    ((2, 3), 64, 0, False)])
def test_stitch_matches_oracle(fpm, grid, side, ov, consistent):
    R, C = grid
    rng = np.random.default_rng(side + ov + 7 * R + C)
    s = side - ov
    if consistent:
        img = rng.standard_normal((R * s + ov, C * s + ov)) + 1j * rng.standard_normal(
            (R * s + ov, C * s + ov)) + 2.0
        fac = np.exp(1j * rng.uniform(-3, 3, (R, C))) * rng.uniform(0.5, 2, (R, C))
        tiles = [[fac[r, c] * img[r * s:r * s + side, c * s:c * s + side] for c in range(C)]
                 for r in range(R)]
    else:
        tiles = [[rng.standard_normal((side, side)) + 1j * rng.standard_normal((side, side)) + 1.5
                  for _ in range(C)] for _ in range(R)]
    tiles = [[t.astype(np.complex64).astype(np.complex128) for t in row] for row in tiles]
    ref = ost.stitch_grid(tiles, ov)
    got = gpu_stitch(fpm, tiles, ov)
    assert got.shape == ref.shape
    assert rel(got, ref) <= TOL
    if consistent:
        assert rel(got, fac[0, 0] * img) <= 1e-5


def test_stitch_host_and_device_agree(fpm):
    rng = np.random.default_rng(3)
    R, C, side, ov = 2, 3, 64, 12
    arr = (rng.standard_normal((R, C, side, side)) + 1j * rng.standard_normal((R, C, side, side))
           + 1.0).astype(np.complex64)
    H, W = fpm.stitched_shape(R, C, side, ov)
    out_h = np.zeros(2 * H * W, np.float32)
    fpm.fpm_stitch(arr.reshape(-1).view(np.float32).copy(), R, C, side, ov, out_h,
                   fpm.FPM_MEM_HOST)
    got = gpu_stitch(fpm, [[arr[r, c] for c in range(C)] for r in range(R)], ov)
    assert np.array_equal(out_h.view(np.complex64).reshape(H, W), got)


def test_stitch_reconstructed_tiles(fpm, orc):
    """A 2 x 2 block of full-field tiles (8 LR px overlap = 32 HR px),
    reconstructed on the GPU and stitched there, against the oracle's
    reconstructions stitched by the oracle."""
    import torch
    tds = fpm_synth.full_fov_tiles(only=[0, 1, 16, 17], iterations=2, schedule=1,
                                   pupil_update=1)
    descs, Is, refs = [], [], []
    for td in tds:
        _, _, I = orc.synthesize(td, z_range=20.0)
        descs.append(td.desc)
        Is.append(I)
        r = orc.reconstruct(td.desc, I)
        refs.append(orc.spectrum_to_object(td.desc, r.S))
    plan = fpm.Plan(descs)
    I = torch.from_numpy(np.concatenate([x.reshape(-1) for x in Is])).cuda()
    obj, _, _ = fpm.device_buffers(plan)
    fpm.fpm_reconstruct(plan, I, fpm.FPM_MEM_DEVICE, obj)
    N = descs[0].N
    ov = 8 * descs[0].upsample
    H, W = fpm.stitched_shape(2, 2, N, ov)
    out = torch.empty(2 * H * W, dtype=torch.float32, device="cuda")
    fpm.fpm_stitch(obj, 2, 2, N, ov, out, fpm.FPM_MEM_DEVICE)
    got = out.cpu().numpy().view(np.complex64).reshape(H, W)
    ref = ost.stitch_grid([[refs[0], refs[1]], [refs[2], refs[3]]], ov)
    assert got.shape == (2 * N - ov, 2 * N - ov)
    assert rel(got, ref) <= 1e-4


def _field(fpm, orc, overlap):
    """Reconstruct the tiles of one shared object on the GPU and stitch them;
    return (stitched field, true field)."""
    import torch
    tds, whole, _ = fpm_synth.shared_object_tiles(tiles_per_side=3, n=64, overlap=overlap,
                                                  iterations=8)
    descs, Is = [], []
    for td in tds:
        d = td.desc
        I = orc.forward(d, orc.object_to_spectrum(d, td.obj))
        Is.append(fpm_synth.poisson_noise(td.rng, I, td.peak_photons))
        descs.append(d)
    plan = fpm.Plan(descs)
    I = torch.from_numpy(np.concatenate([x.reshape(-1) for x in Is])).cuda()
    obj, _, _ = fpm.device_buffers(plan)
    fpm.fpm_reconstruct(plan, I, fpm.FPM_MEM_DEVICE, obj)
    N = descs[0].N
    ov = overlap * descs[0].upsample
    H, W = fpm.stitched_shape(3, 3, N, ov)
    out = torch.empty(2 * H * W, dtype=torch.float32, device="cuda")
    fpm.fpm_stitch(obj, 3, 3, N, ov, out, fpm.FPM_MEM_DEVICE)
    return out.cpu().numpy().view(np.complex64).reshape(H, W).astype(np.complex128), whole


def test_overlap_removes_tile_discontinuities(fpm, orc):
    """Synthetic analogue of Sec. 4.2 / Fig. 11: tiles of one object, each
    reconstructed on its own (each with its own global phase).  Stitched with
    an 8-px overlap (Eq. (1)), the field matches the object up to one global
    complex factor; abutting tiles without overlap keep their separate
    phases, and the error is several times larger."""
    errs = {}
    for ov in (8, 0):
        got, truth = _field(fpm, orc, ov)
        assert got.shape == truth.shape
        c = np.vdot(got, truth) / np.vdot(got, got)   # best single global factor
        errs[ov] = rel(c * got, truth)
    print("field error with overlap %.3e, without %.3e" % (errs[8], errs[0]))
    assert errs[8] < 0.5 * errs[0]
