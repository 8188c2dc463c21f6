"""Host-side checks of the Python binding's buffer marshalling (no GPU
needed): a buffer of the wrong type or too few elements is refused before
the library is called, since the library reads and writes exactly the plan's
element counts and cannot see a Python buffer's size."""
import numpy as np
import pytest

import fpm_synth


@pytest.fixture(scope="module")
def fpm():
    import paper_2203_02507_amd as fpm
    return fpm


@pytest.fixture(scope="module")
def plan(fpm):
    d = fpm_synth.TileDesc(n=64, upsample=2, led_rows=5, led_cols=5, iterations=2)
    return fpm.Plan([d, d])


def intensity(plan, dtype=np.float32, short=0):
    return np.ones(plan.total_intensity - short, dtype)


def test_plan_element_counts(plan):
    assert plan.total_intensity == 2 * 25 * 64 * 64
    assert plan.total_object == 2 * 128 * 128
    assert plan.total_pupil == 2 * 64 * 64
    assert plan.total_residual == 2 * 2


def test_wrong_dtype_refused(fpm, plan):
    with pytest.raises(TypeError, match="intensity"):
        fpm.fpm_reconstruct(plan, intensity(plan, np.float64), fpm.FPM_MEM_HOST)
    obj = np.zeros(plan.total_object, np.complex128)
    with pytest.raises(TypeError, match="object_out"):
        fpm.fpm_reconstruct(plan, intensity(plan), fpm.FPM_MEM_HOST, obj)
    res = np.zeros(plan.total_residual, np.float32)
    with pytest.raises(TypeError, match="residual_out"):
        fpm.fpm_reconstruct(plan, intensity(plan), fpm.FPM_MEM_HOST, None, None, res)


def test_short_buffer_refused(fpm, plan):
    with pytest.raises(ValueError, match="intensity"):
        fpm.fpm_reconstruct(plan, intensity(plan, short=1), fpm.FPM_MEM_HOST)
    # a complex buffer as interleaved float32 needs two floats per element
    obj = np.zeros(plan.total_object, np.float32)
    with pytest.raises(ValueError, match="object_out"):
        fpm.fpm_reconstruct(plan, intensity(plan), fpm.FPM_MEM_HOST, obj)
    pup = np.zeros(plan.total_pupil - 1, np.complex64)
    with pytest.raises(ValueError, match="pupil_out"):
        fpm.fpm_reconstruct(plan, intensity(plan), fpm.FPM_MEM_HOST, None, pup)
    # one LED's images of every tile: sum of n^2 floats
    with pytest.raises(ValueError, match="intensity"):
        fpm.fpm_online_push(plan, 0, np.ones(plan.total_pupil - 1, np.float32), fpm.FPM_MEM_HOST)
    with pytest.raises(ValueError, match="object"):
        fpm.fpm_forward(plan, np.zeros(plan.total_object - 1, np.complex64), None,
                        np.zeros(plan.total_intensity, np.float32), fpm.FPM_MEM_HOST)


def test_stitch_buffers_checked(fpm):
    rows, cols, side, ov = 2, 3, 32, 4
    H, W = fpm.stitched_shape(rows, cols, side, ov)
    tiles = np.zeros((rows, cols, side, side), np.complex64)
    with pytest.raises(ValueError, match="out"):
        fpm.fpm_stitch(tiles, rows, cols, side, ov, np.zeros(H * W - 1, np.complex64),
                       fpm.FPM_MEM_HOST)
    with pytest.raises(TypeError, match="tiles"):
        fpm.fpm_stitch(tiles.astype(np.complex128), rows, cols, side, ov,
                       np.zeros(H * W, np.complex64), fpm.FPM_MEM_HOST)


def test_placement_checked(fpm, plan):
    with pytest.raises(ValueError, match="host memory"):
        fpm.fpm_reconstruct(plan, intensity(plan), fpm.FPM_MEM_DEVICE)
