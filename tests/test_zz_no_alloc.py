"""The allocation-free stitch entry point (fpm_stitch_noalloc) through the C
ABI: the same bits as fpm_stitch on the same device buffers, on two calls in
a row (the second on a smaller grid, so stale scratch from the first would
show), checked against the FP64 stitching oracle too, and the grid limit of
its fixed scratch rejected as an argument error.  Runs last: it shares the
library's per-device scratch with nothing else."""
import numpy as np
import pytest

from oracle import stitch as ost

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fpm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2203_02507_amd as fpm
    return fpm


def _tiles(rng, R, C, side, ov):
    s = side - ov
    img = rng.standard_normal((R * s + ov, C * s + ov)) + 1j * rng.standard_normal(
        (R * s + ov, C * s + ov)) + 2.0
    fac = np.exp(1j * rng.uniform(-3, 3, (R, C))) * rng.uniform(0.5, 2, (R, C))
    return [[(fac[r, c] * img[r * s:r * s + side, c * s:c * s + side]).astype(np.complex64)
             for c in range(C)] for r in range(R)]


def test_noalloc_stitch_equals_stitch(fpm):
    import torch
    rng = np.random.default_rng(20305)
    # the second call is smaller: any scratch word it read without writing
    # first would come from the larger first call and change its result
    for R, C, side, ov in ((6, 7, 64, 10), (2, 3, 96, 16)):
        tiles = _tiles(rng, R, C, side, ov)
        arr = np.stack([np.stack(r) for r in tiles])
        src = torch.from_numpy(arr.reshape(-1).view(np.float32)).cuda()
        H, W = fpm.stitched_shape(R, C, side, ov)
        out_a = torch.full((2 * H * W,), float("nan"), dtype=torch.float32, device="cuda")
        out_b = torch.full((2 * H * W,), float("nan"), dtype=torch.float32, device="cuda")
        print(f"grid {R}x{C} side {side} overlap {ov}", flush=True)
        fpm.fpm_stitch(src, R, C, side, ov, out_a, fpm.FPM_MEM_DEVICE)
        fpm.fpm_stitch_noalloc(src, R, C, side, ov, out_b)
        torch.cuda.synchronize()
        a = out_a.cpu().numpy().view(np.complex64).reshape(H, W)
        b = out_b.cpu().numpy().view(np.complex64).reshape(H, W)
        assert np.array_equal(a, b)
        ref = ost.stitch_grid([[t.astype(np.complex128) for t in row] for row in tiles], ov)
        assert float(np.linalg.norm(b - ref) / np.linalg.norm(ref)) <= 1e-6


def test_noalloc_stitch_rejects_grid_beyond_its_scratch(fpm):
    import torch
    side, ov, R, C = 4, 0, 65, 64  # 4160 tiles > 4096
    src = torch.zeros(2 * R * C * side * side, dtype=torch.float32, device="cuda")
    H, W = fpm.stitched_shape(R, C, side, ov)
    out = torch.zeros(2 * H * W, dtype=torch.float32, device="cuda")
    with pytest.raises(fpm.FpmError) as e:
        fpm.fpm_stitch_noalloc(src, R, C, side, ov, out)
    assert e.value.status == fpm.FPM_E_ARG
    assert "4096" in str(e.value)
    assert bool(torch.all(out == 0))
