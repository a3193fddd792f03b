"""The allocation-free distance transform (lbm_prep_distance_noalloc) against the allocating one
(lbm_prep_distance), through the C-ABI: two calls in a row on the same GPU, the second on a
smaller image (so it runs on what the first left in the shared scratch), both rows-of-whole-
bytes and ragged rows, periodic and walled axes; integer output, so bit-exact. Also: an image
beyond the scratch is refused before anything runs."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lbm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2007_12266_amd import lbm as mod
    mod.load_library()
    return mod


def test_noalloc_distance_equals_the_allocating_call_twice(lbm):
    torch.cuda.set_device(0)
    rng = np.random.default_rng(17)
    cases = [((60, 44, 128), (True, False, True), 2, 0.02),   # rows of whole bytes (wide pack)
             ((21, 13, 37), (False, True, False), 5, 0.1)]    # ragged rows, walls in x and z
    stream = torch.cuda.current_stream()
    for shape, periodic, walls, frac in cases:
        print("noalloc case", shape, periodic, walls, flush=True)
        feature = (rng.random(shape) < frac).astype(np.uint8)
        ref = lbm.prep_distance(feature, periodic, wall_axes=walls)
        f_dev = torch.from_numpy(feature).cuda()
        out = torch.full(shape, 7, dtype=torch.int32, device="cuda")
        lbm.prep_distance_noalloc(f_dev, out, periodic, wall_axes=walls,
                                  stream=stream.cuda_stream)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), ref), shape
    # A no-feature image: every distance is -1 ("none"), like the allocating call.
    empty = torch.zeros((5, 6, 7), dtype=torch.uint8, device="cuda")
    out = torch.empty((5, 6, 7), dtype=torch.int32, device="cuda")
    lbm.prep_distance_noalloc(empty, out, (True, True, True), stream=stream.cuda_stream)
    torch.cuda.synchronize()
    assert (out.cpu().numpy() == -1).all()


def test_noalloc_distance_refuses_an_image_beyond_its_scratch(lbm):
    L = lbm.load_library()
    per = (ctypes.c_int32 * 3)(1, 1, 1)
    st = L.lbm_prep_distance_noalloc(160, 160, 160, per, 0, ctypes.c_void_p(256),
                                     ctypes.c_void_p(256), None)
    assert st == lbm.LBM_ERR_ARG and b"too large" in L.lbm_last_error()
