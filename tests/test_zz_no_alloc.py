"""ccl_label_noalloc (the entry point that allocates nothing, its workspace a
static device array) against ccl_label_ex, the entry point it varies, called
through the C ABI: bit-exact labels and counts on consecutive calls that
share the array, the second with a smaller image, plus the size limit."""
import ctypes
import sys

import numpy as np
import pytest
import torch

from paper_1606_05973_amd import inputs

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def ccl():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1606_05973_amd import ccl as mod
    return mod


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _both(ccl, img, conn):
    """(labels, K) from ccl_label_noalloc and from ccl_label_ex on one image."""
    H, W = img.shape
    stride = img.stride(0)
    stream = torch.cuda.current_stream().cuda_stream or None
    out_n = torch.full((H, W), -7, dtype=torch.int32, device=DEV)
    out_e = torch.full((H, W), -9, dtype=torch.int32, device=DEV)
    k_n = torch.full((1,), -1, dtype=torch.int32, device=DEV)
    k_e = torch.full((1,), -1, dtype=torch.int32, device=DEV)
    st = ccl._lib.ccl_label_noalloc(img.data_ptr(), H, W, stride, conn, out_n.data_ptr(), k_n.data_ptr(), stream)
    assert st == 0, ccl.strerror(st)
    st = ccl._lib.ccl_label_ex(img.data_ptr(), H, W, stride, conn, out_e.data_ptr(), k_e.data_ptr(), 0, stream)
    assert st == 0, ccl.strerror(st)
    torch.cuda.synchronize()
    return out_n.cpu().numpy(), int(k_n.item()), out_e.cpu().numpy(), int(k_e.item())


def _same(ccl, img, conn, what):
    say(f"noalloc case {what} shape={tuple(img.shape)} conn={conn}")
    got, k, ref, kref = _both(ccl, img, conn)
    if not np.array_equal(got, ref):
        bad = np.argwhere(got != ref)
        r, c = bad[0]
        raise AssertionError(f"{what}: {len(bad)} pixels differ; first at {(r, c)} noalloc={got[r, c]} "
                             f"ccl_label_ex={ref[r, c]}")
    assert k == kref and k > 0, (what, k, kref)


def test_noalloc_two_calls_second_smaller(ccl):
    # the second call reuses the array the first one filled, on a smaller
    # image with a ragged tail and a row pitch larger than its width
    big = inputs.bernoulli(3001, 2499, 0.5, seed=11, device=DEV)
    _same(ccl, big, 8, "3001x2499 p=0.5 (first call)")
    small_full = inputs.bernoulli(517, 900, 0.45, seed=12, device=DEV)
    small = small_full[:, :777]
    _same(ccl, small, 4, "517x777 in a 900-byte pitch, p=0.45 (second call, smaller)")


def test_noalloc_largest_fitting_image(ccl):
    # 4096^2 at 4-connectivity is the largest square the static scratch holds
    n = 4096
    need = ccl._lib.ccl_workspace_bytes(n, n, 4)
    assert 0 < need <= ccl.NOALLOC_SCRATCH_BYTES
    img = inputs.bernoulli(n, n, 0.593, seed=13, device=DEV)
    _same(ccl, img, 4, "4096x4096 p=0.593 conn 4")
    _same(ccl, inputs.bernoulli(64, 64, 0.5, seed=14, device=DEV), 8, "64x64 after the largest")


def test_noalloc_rejects_images_beyond_the_scratch(ccl):
    H, W = 8192, 8192
    assert ccl._lib.ccl_workspace_bytes(H, W, 8) > ccl.NOALLOC_SCRATCH_BYTES
    img = torch.zeros((H, W), dtype=torch.uint8, device=DEV)
    out = torch.full((H, W), -5, dtype=torch.int32, device=DEV)
    st = ccl._lib.ccl_label_noalloc(img.data_ptr(), H, W, W, 8, out.data_ptr(), None, None)
    assert st == ccl.STATUS["CCL_ERR_SCRATCH"]
    torch.cuda.synchronize()
    assert bool((out == -5).all())  # nothing launched
    with pytest.raises(ccl.CCLError):
        ccl.label_noalloc(img, 8, out)
