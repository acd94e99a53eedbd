"""Parity of the HIP library against the CPU oracle: bit-exact int32 labels
and component counts on the same seeded bytes, called through the C ABI.

Small and medium sizes span several tiles and ragged tails; the full-size
workloads (21568^2, 16384^2, 20000^2) are compared element by element too,
since the C oracle labels them in seconds."""
import sys

import numpy as np
import pytest
import torch

import oracle
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


def run(ccl, img_dev, conn, tile=0):
    k = torch.full((1,), -1, dtype=torch.int32, device=DEV)
    lab = ccl.label(img_dev, conn=conn, tile=tile, num_components=k)
    torch.cuda.synchronize()
    return lab.cpu().numpy(), int(k.item())


def check(ccl, img_dev, conn, tile=0, what=""):
    say(f"case {what} shape={tuple(img_dev.shape)} conn={conn} tile={tile}")
    got, k = run(ccl, img_dev, conn, tile)
    ref, kref = oracle.cclremsp(img_dev.cpu().numpy(), conn)
    if not np.array_equal(got, ref):
        bad = np.argwhere(got != ref)
        r, c = bad[0]
        raise AssertionError(f"{what}: {len(bad)} pixels differ; first at {(r, c)} gpu={got[r, c]} "
                             f"oracle={ref[r, c]}")
    assert k == kref, (what, k, kref)
    return got, k


def test_config0_512_bernoulli(ccl):
    img = inputs.bernoulli(512, 512, 0.5, seed=0, device=DEV)
    check(ccl, img, 8, what="512x512 p=0.5 seed 0")


SMALL = [(1, 1), (1, 300), (300, 1), (2, 2), (31, 255), (33, 257), (32, 256), (64, 512), (65, 513),
         (100, 1000), (257, 1031), (999, 1000)]


@pytest.mark.parametrize("shape", SMALL)
@pytest.mark.parametrize("conn", [8, 4])
def test_random_shapes(ccl, shape, conn):
    H, W = shape
    for p in (0.1, 0.5, 0.9):
        img = inputs.bernoulli(H, W, p, seed=H * 7 + W, device=DEV)
        check(ccl, img, conn, what=f"bernoulli p={p}")


@pytest.mark.parametrize("conn", [8, 4])
def test_every_tile_shape(ccl, conn):
    img = inputs.bernoulli(700, 900, 0.45, seed=3, device=DEV)
    ref = None
    for tile in range(0, len(ccl.tile_configs()) + 1):
        got, _ = check(ccl, img, conn, tile=tile, what="tile sweep")
        if ref is None:
            ref = got
        assert np.array_equal(got, ref)


@pytest.mark.parametrize("name", inputs.ADVERSARIAL)
def test_every_tile_shape_adversarial(ccl, name):
    """Worst-case node and contact counts (checkerboard, stripes, combs) in
    every tile configuration, including the ones that run 1024 threads."""
    img = inputs.adversarial(name, 600, 1100, device=DEV)
    for tile in range(1, len(ccl.tile_configs()) + 1):
        for conn in (8, 4):
            check(ccl, img, conn, tile=tile, what=f"{name} tile sweep")


def test_region_corner_diagonals(ccl):
    """Pixel pairs that touch only diagonally across every point (32 i, 128 j):
    the corners of the boundary merge's tile regions (whose heights are
    multiples of 32 rows and widths multiples of 128 columns) lie on that
    lattice in every tile configuration, so the contacts across region
    corners, which neither region unites on its own, are all exercised."""
    H, W = 600, 1100
    a = np.zeros((H, W), dtype=np.uint8)
    for y in range(32, H, 32):
        for x in range(128, W, 128):
            if (y // 32 + x // 128) % 2:
                a[y - 1, x - 1] = a[y, x] = 1      # down-right across the corner
            else:
                a[y - 1, x] = a[y, x - 1] = 1      # down-left across the corner
    img = torch.from_numpy(a).to(DEV)
    for tile in range(1, len(ccl.tile_configs()) + 1):
        for conn in (8, 4):
            check(ccl, img, conn, tile=tile, what=f"corner diagonals tile {tile}")


@pytest.mark.parametrize("p", [0.3, 0.407, 0.593, 0.7])
def test_percolation_and_grf(ccl, p):
    img = inputs.bernoulli(1024, 1536, p, seed=11, device=DEV)
    for conn in (8, 4):
        check(ccl, img, conn, what=f"p={p}")
    g = inputs.grf(777, 1111, sigma=2 + 10 * p, q=p, seed=5, device=DEV)
    for conn in (8, 4):
        check(ccl, g, conn, what=f"grf sigma={2 + 10 * p} q={p}")


@pytest.mark.parametrize("name", inputs.ADVERSARIAL)
def test_adversarial_medium(ccl, name):
    img = inputs.adversarial(name, 1000, 1300, device=DEV)
    for conn in (8, 4):
        check(ccl, img, conn, what=name)


def _dense_run_mix(H, W, seed):
    """Noise with vertical 1-px stripes in some tile-sized blocks: tiles whose
    run count exceeds the compact scan's node capacity (stripes: every other
    column starts a run in every row) beside tiles it holds (noise), so that
    both tile-scan forms write tables of one image and the merge joins them."""
    img = inputs.bernoulli(H, W, 0.5, seed=seed, device=DEV)
    cols = torch.arange(W, device=DEV)
    stripe = ((cols % 2) == 0).to(torch.uint8)
    for (r0, c0) in ((0, 0), (64, 256), (128, 700), (200, 1400), (320, 128)):
        img[r0:r0 + 96, c0:c0 + 300] = stripe[c0:c0 + 300]
    # a stripe block with a noise row through it joins the stripes together
    img[150, :] = 1
    return img


def test_compact_and_full_tile_scans_in_one_image(ccl):
    img = _dense_run_mix(420, 1777, 21)
    for conn in (8, 4):
        for tile in (0, 1, 4, 5, 7):
            check(ccl, img, conn, tile=tile, what=f"stripes+noise tile {tile}")
    # a checkerboard block: 4-connectivity makes every pixel a run
    img2 = inputs.bernoulli(333, 999, 0.45, seed=22, device=DEV)
    rr = torch.arange(333, device=DEV)[:, None]
    cc = torch.arange(999, device=DEV)[None, :]
    board = (((rr + cc) % 2) == 0).to(torch.uint8)
    img2[40:200, 100:700] = board[40:200, 100:700]
    for conn in (4, 8):
        check(ccl, img2, conn, what="checkerboard block in noise")


def test_strided_unaligned_and_odd_width(ccl):
    base = inputs.bernoulli(300, 1100, 0.5, seed=9, device=DEV)
    view = base[:, 3:1000]  # 3-byte offset: unaligned rows, stride 1100, W = 997
    for conn in (8, 4):
        check(ccl, view, conn, what="unaligned view")
    narrow = inputs.bernoulli(257, 37, 0.6, seed=2, device=DEV, stride=64)
    for conn in (8, 4):
        check(ccl, narrow, conn, what="stride 64, W 37")


@pytest.mark.parametrize("shape", [(285, 700), (31, 256), (33, 260), (65, 516), (100, 1000), (70, 73)])
def test_no_writes_outside_labels(ccl, shape):
    """The label array is written exactly: a guard band after it (and the
    rows below a ragged last tile row) stays untouched."""
    H, W = shape
    img = inputs.bernoulli(H, W, 0.5, seed=H + W, device=DEV)
    for conn in (8, 4):
        # offset 0: 16-byte aligned rows when W % 4 == 0 (vector stores);
        # offset 1: the label array starts 4 bytes into the buffer (plain stores)
        for off in (0, 1):
            guard = 1 << 20
            big = torch.full((off + H * W + guard,), -7, dtype=torch.int32, device=DEV)
            out = big[off:off + H * W].view(H, W)
            say(f"case guard band shape={shape} conn={conn} offset={off}")
            ccl.label(img, conn, out=out)
            torch.cuda.synchronize()
            ref, _ = oracle.cclremsp(img.cpu().numpy(), conn)
            assert np.array_equal(out.cpu().numpy(), ref)
            assert bool((big[:off] == -7).all()) and bool((big[off + H * W:] == -7).all())


@pytest.mark.parametrize("W", [(1 << 22), (1 << 22) + 4, (1 << 22) + 1])
def test_very_wide_rows(ccl, W):
    """Rows up to 4 Mi pixels take the buffer-store forms of the labeling
    pass, wider rows the plain stores; all must agree with the oracle."""
    img = inputs.bernoulli(3, W, 0.5, seed=W, device=DEV)
    for conn in (8, 4):
        check(ccl, img, conn, what=f"very wide W={W}")


def test_nonzero_bytes_are_foreground(ccl):
    g = torch.Generator().manual_seed(0)
    vals = torch.randint(0, 256, (200, 333), generator=g, dtype=torch.int32)
    vals[vals < 128] = 0
    img = vals.to(torch.uint8).to(DEV)
    for conn in (8, 4):
        check(ccl, img, conn, what="byte values 0..255")


def test_repeatable_and_out_buffer_reuse(ccl):
    img = inputs.bernoulli(640, 480, 0.5, seed=21, device=DEV)
    out = torch.full((640, 480), 12345, dtype=torch.int32, device=DEV)
    a = ccl.label(img, 8, out=out).clone()
    b = ccl.label(img, 8, out=out)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_batch_matches_single(ccl):
    specs = inputs.batch_specs(24, seed=7, max_side=700)
    imgs = [inputs.make(s, device=DEV) for s in specs]
    conns = [8 if i % 3 else 4 for i in range(len(imgs))]
    k = torch.full((len(imgs),), -1, dtype=torch.int32, device=DEV)
    say(f"case batch n={len(imgs)}")
    outs = ccl.label_batch(imgs, conn=conns, num_components=k)
    torch.cuda.synchronize()
    for i, img in enumerate(imgs):
        ref, kref = oracle.cclremsp(img.cpu().numpy(), conns[i])
        assert np.array_equal(outs[i].cpu().numpy(), ref), i
        assert int(k[i].item()) == kref
        single = ccl.label(img, conns[i])
        assert torch.equal(single, outs[i])


def test_batch_mixed_store_forms(ccl):
    """One launch group whose images need different labeling-pass store
    forms: rows of W % 4 == 0 into 16-byte aligned labels (16-byte stores),
    odd widths and a label buffer at a 4-byte offset (4-byte stores), each
    tile taking its own image's form."""
    shapes = [(700, 1024), (333, 517), (640, 768), (129, 250), (513, 1283), (256, 512)]
    imgs = [inputs.bernoulli(H, W, 0.5, seed=40 + i, device=DEV) for i, (H, W) in enumerate(shapes)]
    outs = [torch.full((H, W), -3, dtype=torch.int32, device=DEV) for H, W in shapes]
    # the third image's labels at a 4-byte offset inside a larger buffer
    H2, W2 = shapes[2]
    big = torch.full((H2 * W2 + 1,), -3, dtype=torch.int32, device=DEV)
    outs[2] = big[1:].view(H2, W2)
    assert outs[2].data_ptr() % 16 != 0
    for conn in (8, 4):
        say(f"case mixed store forms conn={conn}")
        ccl.label_batch(imgs, conn=conn, outs=outs)
        torch.cuda.synchronize()
        for i, img in enumerate(imgs):
            ref, _ = oracle.cclremsp(img.cpu().numpy(), conn)
            assert np.array_equal(outs[i].cpu().numpy(), ref), (conn, i)
        assert int(big[0].item()) == -3


def test_empty_batch_and_single_pixel(ccl):
    assert ccl.label_batch([]) == []
    for v in (0, 1):
        img = torch.full((1, 1), v, dtype=torch.uint8, device=DEV)
        got, k = run(ccl, img, 8)
        assert got[0, 0] == v and k == v


# ---------------------------------------------------------------- full size
def test_full_21568_bernoulli_8conn(ccl):
    img = inputs.bernoulli(21568, 21568, 0.5, seed=0, device=DEV)
    check(ccl, img, 8, what="21568^2 p=0.5")


def test_full_21568_percolation_4conn(ccl):
    img = inputs.bernoulli(21568, 21568, 0.593, seed=1, device=DEV)
    check(ccl, img, 4, what="21568^2 p=0.593")


def test_full_16384_grf(ccl):
    img = inputs.grf(16384, 16384, 8.0, 0.5, seed=2, device=DEV)
    check(ccl, img, 8, what="16384^2 grf sigma 8")


# The remaining densities of the single-image configuration, including the
# 8-connectivity percolation threshold (p = 0.407) where a missing barrier in
# the component-label kernel once showed as a few wrong pixels.
@pytest.mark.parametrize("side,p,conn", [(21568, 0.1, 8), (21568, 0.3, 8), (21568, 0.407, 8), (21568, 0.9, 8),
                                         (21568, 0.407, 4), (16384, 0.5, 8), (16384, 0.5, 4)])
def test_full_size_bernoulli(ccl, side, p, conn):
    img = inputs.bernoulli(side, side, p, seed=3, device=DEV)
    check(ccl, img, conn, what=f"{side}^2 p={p}")


@pytest.mark.parametrize("sigma", [2.0, 32.0])
@pytest.mark.parametrize("q", [0.3, 0.7])
def test_full_16384_grf_range(ccl, sigma, q):
    img = inputs.grf(16384, 16384, sigma, q, seed=4, device=DEV)
    for conn in (8, 4):
        check(ccl, img, conn, what=f"16384^2 grf sigma={sigma} q={q}")


@pytest.mark.parametrize("name", ["ones", "zeros", "hstripes", "vstripes"])
def test_full_20000_constant_and_stripes(ccl, name):
    """The longest cross-tile merge chains (one component over the whole
    image) and the tallest / widest components, with their closed-form K."""
    img = inputs.adversarial(name, 20000, 20000, device=DEV)
    expect = {"ones": 1, "zeros": 0, "hstripes": 10000, "vstripes": 10000}[name]
    for conn in (8, 4):
        got, k = check(ccl, img, conn, what=f"20000^2 {name}")
        assert k == expect
        if name == "ones":
            assert got.min() == 1 and got.max() == 1
        if name == "hstripes":
            assert got[::2, :].min() == 1 and got[-2, 0] == 10000 and not got[1::2, :].any()


def test_plain_boundary_calls(ccl):
    """ccl_label and ccl_label_batch called with exactly their contract
    signatures (seven-field descriptors) on real images."""
    import ctypes
    lib = ccl._lib
    imgs = [inputs.bernoulli(517, 1030, 0.45, seed=1, device=DEV),
            inputs.grf(300, 257, 5.0, 0.5, seed=2, device=DEV),
            inputs.adversarial("spiral", 199, 333, device=DEV),
            inputs.bernoulli(64, 4096, 0.6, seed=3, device=DEV)]
    conns = [8, 4, 8, 4]
    for img, conn in zip(imgs, conns):
        say(f"case ccl_label shape={tuple(img.shape)} conn={conn}")
        out = torch.full(tuple(img.shape), -9, dtype=torch.int32, device=DEV)
        H, W = img.shape
        assert lib.ccl_label(img.data_ptr(), H, W, img.stride(0), conn, out.data_ptr(), None) == 0
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), oracle.cclremsp(img.cpu().numpy(), conn)[0])
    say("case ccl_label_batch plain descriptors")
    outs = [torch.full(tuple(im.shape), -9, dtype=torch.int32, device=DEV) for im in imgs]
    k = torch.full((len(imgs),), -1, dtype=torch.int32, device=DEV)
    arr = (ccl.ImageDesc * len(imgs))()
    for i, (img, conn) in enumerate(zip(imgs, conns)):
        arr[i].img = img.data_ptr()
        arr[i].H, arr[i].W = img.shape
        arr[i].stride = img.stride(0)
        arr[i].conn = conn
        arr[i].labels = outs[i].data_ptr()
        arr[i].num_components = k.data_ptr() + 4 * i if i != 2 else None
    need = lib.ccl_workspace_bytes(517, 1030, 8)
    assert need > 0 and lib.ccl_reserve(need, None) == 0
    assert lib.ccl_label_batch(arr, len(imgs), None) == 0
    torch.cuda.synchronize()
    for i, (img, conn) in enumerate(zip(imgs, conns)):
        ref, kref = oracle.cclremsp(img.cpu().numpy(), conn)
        assert np.array_equal(outs[i].cpu().numpy(), ref), i
        assert int(k[i].item()) == (kref if i != 2 else -1)
    assert lib.ccl_strerror(0) == b"success"


def test_binding_rejects_wrong_output_buffers(ccl):
    img = inputs.bernoulli(40, 50, 0.5, seed=1, device=DEV)
    good = torch.empty((40, 50), dtype=torch.int32, device=DEV)
    bad_outs = [torch.empty((40, 51), dtype=torch.int32, device=DEV),
                torch.empty((40, 50), dtype=torch.int64, device=DEV),
                torch.empty((50, 40), dtype=torch.int32, device=DEV).t(),
                torch.empty((40, 50), dtype=torch.int32)]
    for bad in bad_outs:
        with pytest.raises(ValueError):
            ccl.label(img, 8, out=bad)
        with pytest.raises(ValueError):
            ccl.label(img, 8, out=bad, scan=ccl.SCAN_ROW)
        with pytest.raises(ValueError):
            ccl.label_batch([img, img], 8, outs=[good, bad])
        with pytest.raises(ValueError):
            ccl.BatchGraph([img, img], 8, outs=[good, bad])
    short = torch.zeros(1, dtype=torch.int32, device=DEV)
    with pytest.raises(ValueError):
        ccl.label_batch([img, img], 8, num_components=short)
    with pytest.raises(ValueError):
        ccl.label_batch([img, img], 8, num_components=torch.zeros(4, dtype=torch.int32, device=DEV)[::2])
    with pytest.raises(ValueError):
        ccl.label(img, 8, num_components=torch.zeros(1, dtype=torch.int64, device=DEV))
    with pytest.raises(ValueError):
        ccl.label_batch([img, img], 8, outs=[good])
    with pytest.raises(ValueError):
        ccl.label_batch([img, img], [8])


@pytest.mark.parametrize("name", ["spiral", "checkerboard", "comb", "diagonal"])
def test_full_20000_adversarial(ccl, name):
    img = inputs.adversarial(name, 20000, 20000, device=DEV)
    for conn in (8, 4):
        got, k = check(ccl, img, conn, what=f"20000^2 {name}")
        if name in ("spiral", "comb"):
            assert k == 1
        if name == "checkerboard":
            assert k == (1 if conn == 8 else 20000 * 20000 // 2)


# ---------------------------------------------------------- fused threshold
@pytest.mark.parametrize("conn", [8, 4])
def test_threshold_levels(ccl, conn):
    """Binarization fused into the image read: foreground iff byte > level,
    against the oracle on the binarized image, on aligned, odd-width and
    strided grayscale images, for levels across both halves of the range."""
    g = inputs.gray(517, 777, 3.0, seed=9, device=DEV)
    base = inputs.gray(300, 1100, 1.5, seed=10, device=DEV)
    strided = base[:, 5:1030]
    host = {id(g): g.cpu().numpy(), id(strided): strided.cpu().numpy()}
    for img in (g, strided):
        for lv in (0, 1, 64, 127, 128, 129, 200, 254, 255):
            say(f"case threshold level={lv} shape={tuple(img.shape)} conn={conn}")
            k = torch.full((1,), -1, dtype=torch.int32, device=DEV)
            got = ccl.label(img, conn, level=lv, num_components=k)
            torch.cuda.synchronize()
            ref, kref = oracle.cclremsp(oracle.binarize(host[id(img)], lv), conn)
            assert np.array_equal(got.cpu().numpy(), ref), lv
            assert int(k.item()) == kref


def test_threshold_batch_per_image_levels(ccl):
    imgs = [inputs.gray(200 + 37 * i, 300 + 11 * i, 2.0 + i, seed=i, device=DEV) for i in range(6)]
    levels = [0, 90, 127, 128, 170, 250]
    conns = [8, 4, 8, 4, 8, 4]
    say("case threshold batch")
    outs = ccl.label_batch(imgs, conns, level=levels)
    torch.cuda.synchronize()
    for img, o, lv, c in zip(imgs, outs, levels, conns):
        ref = oracle.label(img.cpu().numpy(), c, level=lv)
        assert np.array_equal(o.cpu().numpy(), ref), (lv, c)


def test_threshold_full_size_im2bw(ccl):
    """A paper-scale grayscale image thresholded at luminance 0.5 (level 127)."""
    img = inputs.gray(16384, 16384, 6.0, seed=3, device=DEV)
    say("case threshold 16384^2 level 127")
    k = torch.full((1,), -1, dtype=torch.int32, device=DEV)
    got = ccl.label(img, 8, level=127, num_components=k)
    torch.cuda.synchronize()
    ref, kref = oracle.cclremsp(oracle.binarize(img.cpu().numpy(), 127), 8)
    assert int(k.item()) == kref
    assert np.array_equal(got.cpu().numpy(), ref)


# ------------------------------------------------------ scan strategy (rows)
def _diag_contact_image(H, W, s):
    """Period of four rows: lone pixels at every fourth column, a full row, an
    empty row, pixels at every other column.  Each lone pixel has foreground
    above-left and above-right but not above, so one column holds two diagonal
    contacts with different upper runs; the full row below joins the lone
    pixels into one long run, so neither contact is its run's first."""
    r = np.arange(H)[:, None] % 4
    c = (np.arange(W)[None, :] - s) % 4
    img = ((r == 0) & (c == 1)) | (r == 1) | ((r == 3) & (c % 2 == 0))
    return img.astype(np.uint8)


@pytest.mark.parametrize("scan", ["pair", "row"])
def test_diagonal_contacts_sharing_a_column(ccl, scan):
    """Two diagonal contacts at one column, at every bit position of a mask
    word (four shifts; partners one column into the neighbouring word at bit 0
    and bit 31), flipped both ways, on ragged widths."""
    sc = ccl.SCAN_PAIR if scan == "pair" else ccl.SCAN_ROW
    for (H, W) in [(133, 333), (70, 1000)]:
        for s in range(4):
            base = _diag_contact_image(H, W, s)
            for flip in (None, 0, 1, (0, 1)):
                a = base if flip is None else np.ascontiguousarray(np.flip(base, flip))
                img = torch.from_numpy(a).to(DEV)
                for conn in (8, 4):
                    say(f"case diagonal pattern scan={scan} shape={(H, W)} shift={s} flip={flip} conn={conn}")
                    k = torch.full((1,), -1, dtype=torch.int32, device=DEV)
                    got = ccl.label(img, conn, num_components=k, scan=sc)
                    torch.cuda.synchronize()
                    ref, kref = oracle.cclremsp(a, conn)
                    assert np.array_equal(got.cpu().numpy(), ref), (H, W, s, flip, conn)
                    assert int(k.item()) == kref


@pytest.mark.parametrize("tile", [0, 3, 6])
def test_one_row_scan_8conn(ccl, tile):
    """The one-row tile scan (runs of single rows, diagonal contacts as
    unions) gives the same labels as the oracle under 8-connectivity."""
    cases = [inputs.bernoulli(H, W, p, seed=H + W, device=DEV)
             for (H, W) in [(1, 300), (31, 255), (65, 513), (999, 1000)] for p in (0.1, 0.5, 0.9)]
    cases.append(inputs.grf(777, 1111, 6.0, 0.4, seed=4, device=DEV))
    cases += [inputs.adversarial(n, 700, 900, device=DEV) for n in inputs.ADVERSARIAL]
    for img in cases:
        say(f"case scan=row tile={tile} shape={tuple(img.shape)}")
        k = torch.full((1,), -1, dtype=torch.int32, device=DEV)
        got = ccl.label(img, 8, tile=tile, num_components=k, scan=ccl.SCAN_ROW)
        torch.cuda.synchronize()
        ref, kref = oracle.cclremsp(img.cpu().numpy(), 8)
        assert np.array_equal(got.cpu().numpy(), ref)
        assert int(k.item()) == kref


def test_one_row_scan_batch_and_full_size(ccl):
    specs = inputs.batch_specs(10, seed=3, max_side=600)
    imgs = [inputs.make(s_, device=DEV) for s_ in specs]
    scans = [ccl.SCAN_ROW if i % 2 else ccl.SCAN_PAIR for i in range(len(imgs))]
    conns = [8, 8, 4, 8, 8, 4, 8, 8, 4, 8]
    say("case scan mix batch")
    outs = ccl.label_batch(imgs, conns, scan=scans)
    torch.cuda.synchronize()
    for img, o, c in zip(imgs, outs, conns):
        assert np.array_equal(o.cpu().numpy(), oracle.label(img.cpu().numpy(), c))
    img = inputs.bernoulli(21568, 21568, 0.5, seed=0, device=DEV)
    say("case scan=row 21568^2")
    got = ccl.label(img, 8, scan=ccl.SCAN_ROW)
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy(), oracle.label(img.cpu().numpy(), 8))


# --------------------------------------------------------------- gray levels
def _gray_check(ccl, img, conn, tile=0, level=0, what=""):
    say(f"case gray {what} shape={tuple(img.shape)} conn={conn} tile={tile} level={level}")
    k = torch.full((1,), -1, dtype=torch.int32, device=DEV)
    got = ccl.label_gray(img, conn, tile=tile, num_components=k, level=level)
    torch.cuda.synchronize()
    host = img.cpu().numpy()
    if level:
        host = np.where(host > level, host, 0).astype(np.uint8)
    ref, kref = oracle.gray(host, conn)
    g = got.cpu().numpy()
    if not np.array_equal(g, ref):
        bad = np.argwhere(g != ref)
        r, c = bad[0]
        raise AssertionError(f"gray {what}: {len(bad)} pixels differ; first at {(r, c)} gpu={g[r, c]} "
                             f"oracle={ref[r, c]}")
    assert int(k.item()) == kref


@pytest.mark.parametrize("conn", [8, 4])
def test_gray_levels_small_and_ragged(ccl, conn):
    """Gray-level labeling against the oracle: few-valued noise (short runs,
    many diagonal contacts), quantized smooth fields (large equal regions
    meeting along long borders), odd and strided shapes, every tile."""
    gen = torch.Generator().manual_seed(3)
    for (H, W) in [(1, 1), (1, 300), (300, 1), (31, 255), (65, 513), (257, 1031)]:
        noise = torch.randint(0, 4, (H, W), generator=gen, dtype=torch.int32).to(torch.uint8).to(DEV)
        _gray_check(ccl, noise, conn, what="values 0..3")
        field = (inputs.gray(H, W, 3.0, seed=H + W, device=DEV) // 48).contiguous()
        _gray_check(ccl, field, conn, what="quantized field")
    big = (inputs.gray(700, 900, 4.0, seed=8, device=DEV) // 40).contiguous()
    for tile in range(0, len(ccl.tile_configs()) + 1):
        _gray_check(ccl, big, conn, tile=tile, what="tile sweep")
    base = (inputs.gray(300, 1100, 2.0, seed=10, device=DEV) // 30).contiguous()
    _gray_check(ccl, base[:, 5:1030], conn, what="strided unaligned")
    _gray_check(ccl, big, conn, level=3, what="level 3")


def test_gray_binary_images_match_binary_labeling(ccl):
    for name in ("spiral", "checkerboard", "comb", "diagonal", "ones", "zeros"):
        img = inputs.adversarial(name, 600, 700, device=DEV)
        for conn in (8, 4):
            say(f"case gray==binary {name} conn={conn}")
            a = ccl.label_gray(img, conn)
            b = ccl.label(img, conn)
            torch.cuda.synchronize()
            assert torch.equal(a, b)


def test_gray_batch_and_full_size(ccl):
    imgs = [(inputs.gray(200 + 37 * i, 300 + 11 * i, 2.0 + i, seed=i, device=DEV) // 32).contiguous()
            for i in range(6)]
    grays = [True, False, True, True, False, True]
    conns = [8, 8, 4, 8, 4, 4]
    say("case gray batch")
    outs = ccl.label_batch(imgs, conns, gray=grays)
    torch.cuda.synchronize()
    for im, o, g, c in zip(imgs, outs, grays, conns):
        host = im.cpu().numpy()
        ref = oracle.gray(host, c)[0] if g else oracle.label(host, c)
        assert np.array_equal(o.cpu().numpy(), ref)
    img = (inputs.gray(16384, 16384, 6.0, seed=5, device=DEV) // 32).contiguous()
    _gray_check(ccl, img, 8, what="16384^2 quantized field")


# ------------------------------------------------------- provisional order
def _prov_ref(ccl, img_host, conn, tile=0, scan=0, gray=False):
    th, tw = ccl.tile_shape(tile, conn, scan, gray)
    block = 2 if (conn == 8 and scan == ccl.SCAN_PAIR and not gray) else 1
    return oracle.provisional(img_host, conn, th, tw, block, gray_levels=gray)


def _prov_check(ccl, img, conn, tile=0, what=""):
    say(f"case provisional {what} shape={tuple(img.shape)} conn={conn} tile={tile}")
    k = torch.full((1,), -1, dtype=torch.int32, device=DEV)
    got = ccl.label_provisional(img, conn, tile=tile, num_components=k)
    torch.cuda.synchronize()
    ref, kref = _prov_ref(ccl, img.cpu().numpy(), conn, tile)
    g = got.cpu().numpy()
    if not np.array_equal(g, ref):
        bad = np.argwhere(g != ref)
        r, c = bad[0]
        raise AssertionError(f"provisional {what}: {len(bad)} pixels differ; first at {(r, c)} gpu={g[r, c]} "
                             f"oracle={ref[r, c]}")
    assert int(k.item()) == kref
    return g, kref


@pytest.mark.parametrize("shape", SMALL)
@pytest.mark.parametrize("conn", [8, 4])
def test_provisional_shapes(ccl, shape, conn):
    """Paper-order labels (the flatten's numbering over tile-major provisional
    labels) equal the oracle's numbering pixel for pixel; they are exactly
    1..K and renumber to the canonical labels."""
    H, W = shape
    for p in (0.1, 0.5, 0.9):
        img = inputs.bernoulli(H, W, p, seed=H * 5 + W, device=DEV)
        got, k = _prov_check(ccl, img, conn, what=f"p={p}")
        if k:
            assert got.max() == k and np.unique(got[got > 0]).size == k
        canon = oracle.cclremsp(img.cpu().numpy(), conn)[0]
        assert np.array_equal(oracle.canonical(got)[0], canon)


@pytest.mark.parametrize("conn", [8, 4])
def test_provisional_every_tile_and_pattern(ccl, conn):
    img = inputs.bernoulli(700, 900, 0.45, seed=3, device=DEV)
    for tile in range(1, len(ccl.tile_configs()) + 1):
        _prov_check(ccl, img, conn, tile=tile, what="tile sweep")
    for name in inputs.ADVERSARIAL:
        _prov_check(ccl, inputs.adversarial(name, 600, 1100, device=DEV), conn, what=name)
    g = inputs.grf(777, 1111, 6.0, 0.4, seed=4, device=DEV)
    _prov_check(ccl, g, conn, what="grf")


def test_provisional_batch_mix(ccl):
    """Provisional and canonical images, scans, gray levels, thresholds and
    per-image tiles in one batch: every image as its own oracle says."""
    specs = inputs.batch_specs(14, seed=12, max_side=700)
    imgs = [inputs.make(s_, device=DEV) for s_ in specs]
    imgs[3] = (inputs.gray(imgs[3].shape[0], imgs[3].shape[1], 3.0, seed=3, device=DEV) // 40).contiguous()
    n = len(imgs)
    conns = [8 if i % 3 else 4 for i in range(n)]
    orders = [ccl.PROVISIONAL if i % 2 else ccl.CANONICAL for i in range(n)]
    scans = [ccl.SCAN_ROW if i in (5, 9) else ccl.SCAN_PAIR for i in range(n)]
    grays = [i == 3 for i in range(n)]
    tiles = [0, 2, 3, 0, 5, 6, 1, 7, 0, 4, 2, 0, 3, 1]
    k = torch.full((n,), -1, dtype=torch.int32, device=DEV)
    say("case provisional batch mix")
    outs = ccl.label_batch(imgs, conns, num_components=k, order=orders, scan=scans, gray=grays, tiles=tiles)
    torch.cuda.synchronize()
    for i, img in enumerate(imgs):
        host = img.cpu().numpy()
        if orders[i] == ccl.PROVISIONAL:
            ref, kref = _prov_ref(ccl, host, conns[i], tiles[i], scans[i], grays[i])
        else:
            ref, kref = (oracle.gray if grays[i] else oracle.cclremsp)(host, conns[i])
        assert np.array_equal(outs[i].cpu().numpy(), ref), i
        assert int(k[i].item()) == kref, i


@pytest.mark.parametrize("side,p,conn", [(21568, 0.5, 8), (16384, 0.593, 4)])
def test_provisional_full_size(ccl, side, p, conn):
    img = inputs.bernoulli(side, side, p, seed=0, device=DEV)
    _prov_check(ccl, img, conn, what=f"{side}^2 p={p}")
