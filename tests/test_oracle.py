"""Pins for the CPU oracle (``oracle/``), checked against what the paper and the
mathematics fix rather than against the oracle itself.

* exhaustive enumeration of every small binary image against an independent
  min-label fixed point (covers every leaf of the Fig. 2 decision tree on a
  2x3 window and every case of Algorithm 6 on 3x3 windows);
* textbook BFS flood fill and scipy.ndimage.label on random images;
* closed-form component counts and labels of structured images;
* hand-derived fixtures in tests/golden (Section III problem statement);
* invariants of Algorithm 2 (p[i] <= i, root = set minimum, partition equals
  an independent disjoint-set forest) and postconditions of Algorithm 3;
* agreement of the three labelings (CCLRemSP, ARemSP, PARemSP for any chunk
  count);
* planted mistakes: a copy of the oracle with a plausible bug must fail the
  exhaustive pin.
"""
import glob
import os
import re
import subprocess
import ctypes

import numpy as np
import pytest
import scipy.ndimage as ndi

import oracle
from paper_1606_05973_amd import inputs
from tests import _pins

SHAPES_FULL = [(1, 1), (1, 7), (7, 1), (2, 3), (3, 2), (3, 3), (2, 7), (4, 4), (3, 5), (5, 3)]
SHAPES_PACKED = [(2, 8), (8, 2), (1, 16), (16, 1), (4, 4)]


@pytest.mark.parametrize("shape", SHAPES_FULL)
@pytest.mark.parametrize("conn", [4, 8])
def test_exhaustive_each_image(shape, conn):
    """Every image of the shape, labelled one call at a time by each variant."""
    H, W = shape
    imgs = _pins.all_images(H, W)
    ref = _pins.min_propagation(imgs, conn)
    for i in range(imgs.shape[0]):
        a, ka = oracle.cclremsp(imgs[i], conn)
        assert np.array_equal(a, ref[i]), (shape, conn, imgs[i])
        assert ka == int(ref[i].max())
    # the two-row scan and its chunked parallel form on a subsample
    step = max(1, imgs.shape[0] // 4096)
    for i in range(0, imgs.shape[0], step):
        b, _ = oracle.aremsp(imgs[i], conn)
        assert np.array_equal(b, ref[i]), (shape, conn, imgs[i])
        c, _ = oracle.paremsp(imgs[i], conn, nchunks=1 + i % 3)
        assert np.array_equal(c, ref[i]), (shape, conn, imgs[i])


def _pack(imgs, gap=1):
    """Tile a stack of small images into one big image with background gutters."""
    N, H, W = imgs.shape
    g = int(np.ceil(np.sqrt(N)))
    big = np.zeros((g * (H + gap), g * (W + gap)), dtype=np.uint8)
    for i in range(N):
        r, c = divmod(i, g)
        big[r * (H + gap):r * (H + gap) + H, c * (W + gap):c * (W + gap) + W] = imgs[i]
    return big, g


def _unpack_canonical(big, N, H, W, g, gap=1):
    """Cut the big labeling into blocks and renumber each block canonically.

    The big labeling is canonical, so inside a block the labels already grow
    with first occurrence; the block's own numbering is the dense rank."""
    blocks = big.reshape(g, H + gap, g, W + gap).transpose(0, 2, 1, 3)[:, :, :H, :W]
    L = blocks.reshape(g * g, H * W)[:N].astype(np.int64)
    key = np.arange(N, dtype=np.int64)[:, None] * (int(L.max()) + 1) + L
    uniq, inv = np.unique(key, return_inverse=True)
    inv = inv.reshape(N, H * W)
    base = np.searchsorted(uniq, np.arange(N, dtype=np.int64) * (int(L.max()) + 1))
    has_zero = (L == 0).any(axis=1)
    rank = inv - base[:, None] + np.where(has_zero, 0, 1)[:, None]
    return np.where(L == 0, 0, rank).reshape(N, H, W).astype(np.int32)


@pytest.mark.parametrize("shape", SHAPES_PACKED)
@pytest.mark.parametrize("conn", [4, 8])
def test_exhaustive_packed(shape, conn):
    """All 2^16 images of 16 pixels, labelled inside one big gutter image."""
    H, W = shape
    imgs = _pins.all_images(H, W)
    ref = _pins.min_propagation(imgs, conn)
    big, g = _pack(imgs)
    for variant in ("cclremsp", "aremsp", "paremsp"):
        if variant == "paremsp":
            lab, _ = oracle.paremsp(big, conn, nchunks=7)
        else:
            lab, _ = getattr(oracle, variant)(big, conn)
        got = _unpack_canonical(lab, imgs.shape[0], H, W, g)
        bad = np.nonzero((got != ref).reshape(len(imgs), -1).any(axis=1))[0]
        assert bad.size == 0, (variant, shape, conn, imgs[bad[0]])


@pytest.mark.parametrize("conn", [4, 8])
def test_bfs_random(conn):
    rng = np.random.default_rng(1234 + conn)
    for _ in range(300):
        H, W = rng.integers(1, 14, size=2)
        img = (rng.random((H, W)) < rng.random()).astype(np.uint8)
        ref = _pins.bfs_labels(img, conn)
        lab, k = oracle.cclremsp(img, conn)
        assert np.array_equal(lab, ref)
        assert k == ref.max()


@pytest.mark.parametrize("conn", [4, 8])
def test_scipy_random(conn):
    """scipy.ndimage.label numbers components in raster order of first pixel."""
    st = np.ones((3, 3), dtype=bool) if conn == 8 else None
    rng = np.random.default_rng(99 + conn)
    cases = []
    for _ in range(40):
        H, W = rng.integers(1, 300, size=2)
        cases.append((rng.random((H, W)) < rng.uniform(0.05, 0.95)).astype(np.uint8))
    for sigma in (1.5, 4.0, 9.0):
        cases.append(inputs.grf(257, 311, sigma, 0.5, seed=int(sigma * 10)).numpy())
    for img in cases:
        ref, k = ndi.label(img, structure=st)
        for fn in (oracle.cclremsp, oracle.aremsp):
            lab, kk = fn(img, conn)
            assert kk == k
            assert np.array_equal(lab, ref)
        lab, kk = oracle.paremsp(img, conn, nchunks=int(rng.integers(1, 12)))
        assert kk == k and np.array_equal(lab, ref)


def _rank_labels(mask):
    """Canonical labels when every foreground pixel is its own component."""
    flat = mask.ravel().astype(np.int64)
    lab = np.cumsum(flat) * flat
    return lab.reshape(mask.shape).astype(np.int32)


SIZES = [(1, 1), (1, 6), (6, 1), (2, 2), (5, 7), (8, 8), (33, 65), (64, 31), (100, 101)]


@pytest.mark.parametrize("H,W", SIZES)
def test_closed_forms(H, W):
    r = np.arange(H)[:, None]
    c = np.arange(W)[None, :]
    for conn in (4, 8):
        # all-zeros: K = 0
        lab, k = oracle.cclremsp(inputs.adversarial("zeros", H, W).numpy(), conn)
        assert k == 0 and not lab.any()
        # all-ones: K = 1, every label 1
        lab, k = oracle.cclremsp(inputs.adversarial("ones", H, W).numpy(), conn)
        assert k == 1 and (lab == 1).all()
        # horizontal stripes on even rows: component r/2 + 1
        img = inputs.adversarial("hstripes", H, W).numpy()
        lab, k = oracle.cclremsp(img, conn)
        assert k == (H + 1) // 2
        assert np.array_equal(lab, np.where(r % 2 == 0, r // 2 + 1, 0) * np.ones_like(c))
        # vertical stripes on even columns: component c/2 + 1
        img = inputs.adversarial("vstripes", H, W).numpy()
        lab, k = oracle.cclremsp(img, conn)
        assert k == (W + 1) // 2
        assert np.array_equal(lab, np.where(c % 2 == 0, c // 2 + 1, 0) * np.ones_like(r))
        # comb: teeth joined by the bottom row -> one component
        img = inputs.adversarial("comb", H, W).numpy()
        lab, k = oracle.cclremsp(img, conn)
        assert k == 1 and np.array_equal(lab, img.astype(np.int32))
        # spiral: one winding component
        img = inputs.adversarial("spiral", H, W).numpy()
        lab, k = oracle.cclremsp(img, conn)
        assert k == 1 and np.array_equal(lab, img.astype(np.int32))
    # checkerboard: one component under 8-connectivity (H, W >= 2),
    # one component per foreground pixel under 4-connectivity
    img = inputs.adversarial("checkerboard", H, W).numpy()
    lab, k = oracle.cclremsp(img, 8)
    if H >= 2 and W >= 2:
        assert k == 1 and np.array_equal(lab, img.astype(np.int32))
    else:
        assert np.array_equal(lab, _rank_labels(img))
    lab, k = oracle.cclremsp(img, 4)
    assert k == int(img.sum()) == (H * W + 1) // 2
    assert np.array_equal(lab, _rank_labels(img))
    if W % 2 == 0:
        assert np.array_equal(lab, np.where(img == 1, (r * W + c) // 2 + 1, 0))
    # diagonal stripes (r + c) % 4 == 0: anti-diagonal j is component j + 1
    # under 8-connectivity, every pixel is alone under 4-connectivity
    img = inputs.adversarial("diagonal", H, W).numpy()
    lab, k = oracle.cclremsp(img, 8)
    assert k == (H + W - 2) // 4 + 1
    assert np.array_equal(lab, np.where(img == 1, (r + c) // 4 + 1, 0))
    lab, k = oracle.cclremsp(img, 4)
    assert k == int(img.sum()) and np.array_equal(lab, _rank_labels(img))


@pytest.mark.parametrize("path", sorted(glob.glob(os.path.join(os.path.dirname(__file__), "golden", "*.txt"))))
def test_golden(path):
    img, expect = _pins.read_golden(path)
    assert expect
    for conn, (lab_ref, k_ref) in expect.items():
        # the fixture itself agrees with the textbook flood fill
        assert np.array_equal(_pins.bfs_labels(img, conn), lab_ref)
        for fn in (oracle.cclremsp, oracle.aremsp):
            lab, k = fn(img, conn)
            assert k == k_ref and np.array_equal(lab, lab_ref), (fn.__name__, conn)
        lab, k = oracle.paremsp(img, conn, nchunks=2)
        assert k == k_ref and np.array_equal(lab, lab_ref)


class _DSU:
    def __init__(self, n):
        self.p = list(range(n))

    def find(self, x):
        while self.p[x] != x:
            self.p[x] = self.p[self.p[x]]
            x = self.p[x]
        return x

    def union(self, a, b):
        self.p[self.find(a)] = self.find(b)


@pytest.mark.parametrize("fn", [oracle.merge_pairs, oracle.merger_pairs])
def test_merge_invariants(fn):
    """Algorithm 2 / 8: p[i] <= i, roots are set minima, partition is right."""
    rng = np.random.default_rng(5)
    for trial in range(200):
        n = int(rng.integers(2, 60))
        m = int(rng.integers(0, 2 * n))
        pairs = rng.integers(0, n, size=(m, 2)).astype(np.int32)
        p = fn(np.arange(n, dtype=np.int32), pairs)
        assert (p <= np.arange(n)).all()
        d = _DSU(n)
        for x, y in pairs:
            d.union(int(x), int(y))

        def root(x):
            while p[x] != x:
                x = p[x]
            return x

        groups = {}
        for i in range(n):
            groups.setdefault(d.find(i), []).append(i)
        for members in groups.values():
            roots = {root(i) for i in members}
            assert roots == {min(members)}


def test_flatten_postconditions():
    """Algorithm 3: consecutive labels 1..K; a root gets 1 + its rank among roots."""
    rng = np.random.default_rng(6)
    for trial in range(200):
        n = int(rng.integers(2, 80))
        pairs = rng.integers(1, n, size=(int(rng.integers(0, n)), 2)).astype(np.int32)
        p = oracle.merge_pairs(np.arange(n, dtype=np.int32), pairs)
        roots = [i for i in range(1, n) if p[i] == i]
        q, k = oracle.flatten(p, n - 1)
        assert k == len(roots)
        assert sorted(set(q[1:].tolist())) == list(range(1, k + 1))
        for rank, r in enumerate(roots):
            assert q[r] == rank + 1
        for i in range(1, n):
            j = i
            while p[j] != j:
                j = p[j]
            assert q[i] == q[j]


def test_variants_agree_chunks():
    """PARemSP gives the same labels for every chunk count (Section IV)."""
    rng = np.random.default_rng(8)
    for trial in range(30):
        H, W = int(rng.integers(1, 90)), int(rng.integers(1, 90))
        img = (rng.random((H, W)) < rng.uniform(0.2, 0.8)).astype(np.uint8)
        for conn in (4, 8):
            ref, k = oracle.cclremsp(img, conn)
            for t in range(1, 9):
                lab, kk = oracle.paremsp(img, conn, nchunks=t)
                assert kk == k and np.array_equal(lab, ref), (H, W, conn, t)


def test_threaded_paremsp_agrees():
    """PARemSP with one thread per chunk (concurrent boundary unions under
    Algorithm 8's locks) gives CCLRemSP's labels for every thread count, on
    random images and on a dense image where many unions race for the same
    large sets."""
    rng = np.random.default_rng(81)
    for trial in range(20):
        H, W = int(rng.integers(1, 120)), int(rng.integers(1, 120))
        img = (rng.random((H, W)) < rng.uniform(0.2, 0.8)).astype(np.uint8)
        for conn in (4, 8):
            ref, k = oracle.cclremsp(img, conn)
            for t in (1, 2, 3, 5, 8, 16):
                lab, kk = oracle.paremsp_threads(img, conn, nthreads=t)
                assert kk == k and np.array_equal(lab, ref), (H, W, conn, t)
    big = (rng.random((600, 700)) < 0.6).astype(np.uint8)
    for conn in (4, 8):
        ref, k = oracle.cclremsp(big, conn)
        for t in (4, 16, 64):
            lab, kk = oracle.paremsp_threads(big, conn, nthreads=t)
            assert kk == k and np.array_equal(lab, ref), (conn, t)


def test_paper_numbering_is_not_canonical():
    """ARemSP's own flatten numbering follows label creation order of the
    two-row scan, which is not raster order; the partition is the same but the
    numbering differs on some images.  This is why the library ranks
    components by smallest raster index instead."""
    rng = np.random.default_rng(3)
    differ = 0
    for _ in range(300):
        img = (rng.random((9, 9)) < 0.5).astype(np.uint8)
        raw, k_raw = oracle.aremsp(img, 8, raw=True)
        ref, k = oracle.cclremsp(img, 8)
        assert k_raw == k
        assert np.array_equal(oracle.canonical(raw)[0], ref)
        differ += not np.array_equal(raw, ref)
    assert differ > 0


def test_oracle_argument_errors():
    img = np.zeros((3, 3), np.uint8)
    with pytest.raises(ValueError):
        oracle.cclremsp(img, 6)
    with pytest.raises(ValueError):
        oracle.cclremsp(np.zeros((0, 3), np.uint8), 8)


def test_strided_input():
    rng = np.random.default_rng(4)
    base = (rng.random((50, 80)) < 0.5).astype(np.uint8)
    view = base[:, 5:70]
    assert view.strides[0] == 80
    ref = _pins.bfs_labels(view, 8)
    assert np.array_equal(oracle.cclremsp(view, 8)[0], ref)


# ---------------------------------------------------------------- mutations
MUTANTS = [
    # drop the merge in copy(c,a): label(e) = p[label(c)]
    ("*e = merge(p, lc, la);        /* copy(c,a) */", "*e = p[lc];"),
    # transposed neighbour: read c at (r-1, c) instead of (r-1, c+1)
    ("int cc = image_at(im, r - 1, c + 1), d", "int cc = image_at(im, r - 1, c), d"),
    # wrong comparison in Rem's link direction (the side with the smaller
    # parent moves)
    ("        if (px == py)\n            return px;\n        if (px < py) {",
     "        if (px == py)\n            return px;\n        if (px > py) {"),
    # flatten treats every label as a root
    ("        if (p[i] < i)\n            p[i] = p[p[i]];", "        if (p[i] < 0)\n            p[i] = p[p[i]];"),
    # 4-connectivity merge dropped
    ("                if (b && d)\n                    *e = merge(p, lb, ld);", "                if (b && d)\n                    *e = p[lb];"),
    # a root is found but never linked (the union is dropped)
    ("        p[x] = py; /* a root is linked, an inner node spliced */\n        if (px == x)\n            return py;",
     "        if (px == x)\n            return py;\n        p[x] = py;"),
]


def _build_mutant(tmp_path, i, old, new):
    src = open(os.path.join(os.path.dirname(oracle.__file__), "ccl_oracle.c")).read()
    assert src.count(old) == 1, old
    mut = tmp_path / f"mutant{i}.c"
    mut.write_text(src.replace(old, new))
    so = tmp_path / f"mutant{i}.so"
    subprocess.run(["gcc", "-O1", "-std=c11", "-pthread", "-shared", "-fPIC", "-o", str(so), str(mut)], check=True)
    lib = ctypes.CDLL(str(so))
    u8p = ctypes.POINTER(ctypes.c_uint8)
    i32p = ctypes.POINTER(ctypes.c_int32)
    lib.oracle_cclremsp.argtypes = [u8p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int, i32p]
    lib.oracle_cclremsp.restype = ctypes.c_int64
    return lib


@pytest.mark.parametrize("i", range(len(MUTANTS)))
def test_planted_mistakes_are_caught(tmp_path, i):
    old, new = MUTANTS[i]
    lib = _build_mutant(tmp_path, i, old, new)
    caught = False
    for conn in (8, 4):
        for shape in ((3, 3), (4, 4)):
            imgs = _pins.all_images(*shape)
            ref = _pins.min_propagation(imgs, conn)
            out = np.empty(shape, np.int32)
            for j in range(imgs.shape[0]):
                img = np.ascontiguousarray(imgs[j])
                lib.oracle_cclremsp(img.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), shape[0], shape[1],
                                    shape[1], conn, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
                if not np.array_equal(out, ref[j]):
                    caught = True
                    break
            if caught:
                break
        if caught:
            break
    assert caught, f"mutant {i} survived the exhaustive pin"


def test_binarize_pins():
    """Section V thresholding: foreground iff byte > level, checked against
    every (byte, level) pair; level 0 is the nonzero test and level 255
    leaves nothing; thresholding then labeling equals labeling a 0/1 image
    built by hand."""
    v = np.arange(256, dtype=np.uint8)
    for lv in range(256):
        b = oracle.binarize(v[None, :], lv)[0]
        assert b.dtype == np.uint8
        assert [int(x) for x in b] == [1 if x > lv else 0 for x in range(256)]
    img = np.array([[0, 200, 90], [130, 127, 128], [255, 1, 0]], dtype=np.uint8)
    # level 127 (a 0.5 luminance threshold): 128, 130, 200, 255 are foreground
    assert oracle.binarize(img, 127).tolist() == [[0, 1, 0], [1, 0, 1], [1, 0, 0]]
    lab = oracle.label(img, 8, level=127)
    assert lab.tolist() == [[0, 1, 0], [1, 0, 1], [1, 0, 0]]
    lab4 = oracle.label(img, 4, level=127)
    assert lab4.tolist() == [[0, 1, 0], [2, 0, 3], [2, 0, 0]]
    assert oracle.label(img, 8, level=0).tolist() == oracle.label((img > 0).astype(np.uint8), 8).tolist()
    assert oracle.label(img, 8, level=255).max() == 0


# ------------------------------------------------------------ gray levels
@pytest.mark.parametrize("conn", [8, 4])
def test_gray_exhaustive(conn):
    """Gray-level oracle against flood fill on every 3x3 image over values
    {0, 1, 2} and every 2x3 image over {0..3}."""
    for shape, levels in (((3, 3), 3), ((2, 3), 4)):
        imgs = _pins.all_gray_images(*shape, levels)
        for j in range(imgs.shape[0]):
            got, k = oracle.gray(imgs[j], conn)
            ref = _pins.bfs_gray_labels(imgs[j], conn)
            assert np.array_equal(got, ref), (shape, j)
            assert k == ref.max()


@pytest.mark.parametrize("conn", [8, 4])
def test_gray_scipy_and_binary(conn):
    """Per-value scipy labeling, renumbered by first raster pixel, equals the
    gray oracle; on 0/1 images the gray oracle is the binary one."""
    import scipy.ndimage as ndi
    rng = np.random.default_rng(5)
    st = np.ones((3, 3)) if conn == 8 else None
    for trial in range(6):
        H, W = rng.integers(20, 90, size=2)
        img = rng.integers(0, 4, size=(H, W)).astype(np.uint8)
        comb = np.zeros((H, W), np.int64)
        base = 0
        for v in range(1, 4):
            lab, n = ndi.label(img == v, structure=st)
            comb[lab > 0] = lab[lab > 0] + base
            base += n
        canon, kk = oracle.canonical(comb.astype(np.int32))
        got, k = oracle.gray(img, conn)
        assert np.array_equal(got, canon) and k == kk
        b = (rng.random((H, W)) < 0.5).astype(np.uint8)
        assert np.array_equal(oracle.gray(b, conn)[0], oracle.cclremsp(b, conn)[0])


def test_gray_closed_form():
    """Columns of distinct values: each column is one component under both
    connectivities (diagonal neighbours differ), label = column + 1."""
    H, W = 17, 200
    img = np.tile((1 + np.arange(W) % 250).astype(np.uint8), (H, 1))
    for conn in (8, 4):
        got, k = oracle.gray(img, conn)
        assert k == W and np.array_equal(got, np.tile(np.arange(1, W + 1, dtype=np.int32), (H, 1)))


GRAY_MUTANTS = [
    # values ignored: any two object neighbours connect
    ("im->img[rr * im->stride + cc] != v)", "im->img[rr * im->stride + cc] == 0)"),
    # only the first equal neighbour is used (no merge)
    ("l = l ? merge(p, l, ln) : p[ln];", "l = l ? l : p[ln];"),
]


@pytest.mark.parametrize("i", range(len(GRAY_MUTANTS)))
def test_gray_planted_mistakes_are_caught(tmp_path, i):
    old, new = GRAY_MUTANTS[i]
    src = open(os.path.join(os.path.dirname(oracle.__file__), "ccl_oracle.c")).read()
    assert src.count(old) == 1, old
    mut = tmp_path / f"gmutant{i}.c"
    mut.write_text(src.replace(old, new))
    so = tmp_path / f"gmutant{i}.so"
    subprocess.run(["gcc", "-O1", "-std=c11", "-pthread", "-shared", "-fPIC", "-o", str(so), str(mut)], check=True)
    lib = ctypes.CDLL(str(so))
    u8p, i32p = ctypes.POINTER(ctypes.c_uint8), ctypes.POINTER(ctypes.c_int32)
    lib.oracle_gray.argtypes = [u8p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int, i32p]
    lib.oracle_gray.restype = ctypes.c_int64
    imgs = _pins.all_gray_images(3, 3, 3)
    out = np.empty((3, 3), np.int32)
    caught = False
    for conn in (8, 4):
        for j in range(imgs.shape[0]):
            img = np.ascontiguousarray(imgs[j])
            lib.oracle_gray(img.ctypes.data_as(u8p), 3, 3, 3, conn, out.ctypes.data_as(i32p))
            if not np.array_equal(out, _pins.bfs_gray_labels(img, conn)):
                caught = True
                break
        if caught:
            break
    assert caught, f"gray mutant {i} survived"


# ------------------------------------------------------- provisional order
ROOT_GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "provisional")


def _read_prov_golden(path):
    """Fixture: a `tile th tw block` line, then image / labels8 / labels4."""
    lines = [l.split() for l in open(path) if l.strip() and not l.lstrip().startswith("#")]
    th, tw, block = (int(v) for v in lines[0][1:4])
    img, out = None, {}
    sec, rows, k = None, [], None
    for l in lines[1:] + [["end"]]:
        if l[0] in ("image", "labels8", "labels4", "end"):
            if sec == "image":
                img = np.array(rows, dtype=np.uint8)
            elif sec:
                out[int(sec[-1])] = (np.array(rows, dtype=np.int32), k)
            sec, rows, k = l[0], [], (int(l[1]) if len(l) > 1 else None)
        else:
            rows.append([int(v) for v in l])
    return img, th, tw, block, out


@pytest.mark.parametrize("name", ["tiles_4x4.txt", "pairs_2x4.txt"])
def test_provisional_golden(name):
    """Hand-derived provisional numberings (tile order, node order inside a
    tile), for the oracle and for the step-by-step reference alike."""
    img, th, tw, block, want = _read_prov_golden(os.path.join(ROOT_GOLDEN, name))
    for conn, (labels, k) in want.items():
        got, kk = oracle.provisional(img, conn, th, tw, block)
        assert np.array_equal(got, labels) and kk == k, (name, conn)
        got2, k2 = _pins.provisional_by_steps(img, conn, th, tw, block)
        assert np.array_equal(got2, labels) and k2 == k, (name, conn)


@pytest.mark.parametrize("conn", [8, 4])
def test_provisional_against_steps(conn):
    """The oracle's provisional numbering (ranking sets by their smallest
    (tile, block row, column)) equals the paper's steps done one by one:
    per-tile labels in node order with per-tile label ranges, unions across
    tile edges, then Algorithm 3's consecutive numbering.  Also: the same
    partition as the canonical labels, labels exactly 1..K."""
    rng = np.random.default_rng(5)
    cases = 0
    for (H, W) in [(1, 9), (7, 1), (6, 9), (9, 14), (13, 11), (16, 16)]:
        for (th, tw) in [(2, 4), (4, 8), (3, 5), (16, 32)]:
            for block in ((1, 2) if conn == 8 else (1,)):
                if th % block:
                    continue
                for p in (0.3, 0.6):
                    img = (rng.random((H, W)) < p).astype(np.uint8)
                    got, k = oracle.provisional(img, conn, th, tw, block)
                    ref, kref = _pins.provisional_by_steps(img, conn, th, tw, block)
                    assert k == kref and np.array_equal(got, ref), (H, W, th, tw, block, p)
                    canon, kc = oracle.cclremsp(img, conn)
                    assert kc == k and np.array_equal(oracle.canonical(got)[0], canon)
                    if k:
                        assert set(np.unique(got[got > 0])) == set(range(1, k + 1))
                    cases += 1
    assert cases >= 48
    # gray levels: runs of equal values in single rows
    for (H, W) in [(8, 10), (12, 7)]:
        img = rng.integers(0, 3, (H, W)).astype(np.uint8)
        got, k = oracle.provisional(img, conn, 4, 4, 1, gray_levels=True)
        ref, kref = _pins.provisional_by_steps(img, conn, 4, 4, 1, gray=True)
        assert k == kref and np.array_equal(got, ref)


def test_provisional_special_cases():
    """One tile and single-row nodes: provisional order is raster order of
    each set's first pixel, i.e. the canonical numbering."""
    rng = np.random.default_rng(9)
    for conn in (8, 4):
        img = (rng.random((40, 50)) < 0.5).astype(np.uint8)
        got, _ = oracle.provisional(img, conn, 64, 64, 1)
        assert np.array_equal(got, oracle.cclremsp(img, conn)[0])
        zeros = np.zeros((5, 7), np.uint8)
        assert oracle.provisional(zeros, conn, 2, 4, 1)[1] == 0
