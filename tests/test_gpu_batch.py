"""Batched, captured and served forms on the GPU, bit-exact against the
oracle and against the single-image path."""
import random
import threading
import time

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


def _oracle(img, conn):
    return oracle.cclremsp(img.cpu().numpy(), conn)


def test_batch_graph_replays(ccl):
    specs = inputs.batch_specs(12, seed=31, max_side=600)
    imgs = [inputs.make(s, device=DEV) for s in specs]
    conns = [8 if i % 2 else 4 for i in range(len(imgs))]
    k = torch.full((len(imgs),), -1, dtype=torch.int32, device=DEV)
    say("case graph create n=12")
    g = ccl.BatchGraph(imgs, conns, num_components=k)
    other = inputs.bernoulli(300, 300, 0.5, seed=5, device=DEV)
    try:
        for rep in range(4):
            # new content in the same buffers, eager work between replays
            for i, (img, s) in enumerate(zip(imgs, specs)):
                img.copy_(inputs.bernoulli(s["H"], s["W"], 0.2 + 0.15 * ((rep + i) % 4), seed=rep * 100 + i,
                                           device=DEV))
            eager = ccl.label(other, 8)
            torch.cuda.synchronize()
            say(f"case graph replay {rep}")
            outs = g.launch()
            torch.cuda.synchronize()
            for i, img in enumerate(imgs):
                ref, kref = _oracle(img, conns[i])
                assert np.array_equal(outs[i].cpu().numpy(), ref), (rep, i)
                assert int(k[i].item()) == kref
            assert torch.equal(eager, ccl.label(other, 8))
    finally:
        g.close()


def test_autotuner_picks_and_caches(ccl, tmp_path):
    from paper_1606_05973_amd import autotune
    t = autotune.Autotuner(str(tmp_path / "tiles.json"))
    say("case autotune 1024x1536")
    tile = t.best_tile(1024, 1536, 8)
    assert 1 <= tile <= len(ccl.tile_configs())
    t2 = autotune.Autotuner(str(tmp_path / "tiles.json"))
    assert t2.best_tile(1024, 1536, 8) == tile  # from the cache
    imgs = [inputs.bernoulli(200 + 37 * i, 300, 0.5, seed=i, device=DEV) for i in range(6)]
    bt = t.tune_batch(imgs, [8] * 6, key="six")
    outs = ccl.label_batch(imgs, 8, tile=bt)
    torch.cuda.synchronize()
    for img, o in zip(imgs, outs):
        assert np.array_equal(o.cpu().numpy(), _oracle(img, 8)[0])
    # the schedule tuner: per-bucket tiles or one tile, whichever is faster
    mix = [inputs.bernoulli(64 + 97 * i, 90 + 211 * (i % 3), 0.5, seed=50 + i, device=DEV) for i in range(7)]
    conns = [8, 4, 8, 8, 4, 8, 4]
    say("case autotune plan_batch n=7")
    plan = t.plan_batch(mix, conns, key="seven")
    assert plan["schedule"] in ("one tile", "per bucket") and len(plan["tiles"]) == len(mix)
    assert all(1 <= x <= len(ccl.tile_configs()) for x in plan["tiles"])
    assert t.plan_batch(mix, conns, key="seven")["tiles"] == plan["tiles"]  # from the cache
    outs = ccl.label_batch(mix, conns, tiles=plan["tiles"])
    g = ccl.BatchGraph(mix, conns, tiles=plan["tiles"])
    try:
        gout = g.launch()
        torch.cuda.synchronize()
        for i, img in enumerate(mix):
            ref = _oracle(img, conns[i])[0]
            assert np.array_equal(outs[i].cpu().numpy(), ref) and np.array_equal(gout[i].cpu().numpy(), ref), i
    finally:
        g.close()


def test_serve_alone_equals_mix(ccl):
    from paper_1606_05973_amd import serve
    rng = random.Random(7)
    pool = []
    for i, s in enumerate(inputs.batch_specs(40, seed=11, max_side=900)):
        pool.append((inputs.make(s, device=DEV), 8 if rng.random() < 0.5 else 4))
    torch.cuda.synchronize()
    srv = serve.Server(hbm_budget=256 << 20, n_streams=3, max_batch=8)
    reqs = []
    say("case serve 120 requests")
    t0 = time.perf_counter()
    for n in range(120):
        img, conn = pool[rng.randrange(len(pool))]
        reqs.append(srv.submit(img, conn))
        if n % 7 == 0:
            time.sleep(rng.random() * 0.002)
    huge = torch.zeros((12000, 12000), dtype=torch.uint8, device=DEV)
    rej = srv.submit(huge, 8)
    srv.drain()
    t1 = time.perf_counter()
    st = srv.stats(t0, t1)
    srv.close()
    say("serve stats", st)
    assert rej.status == "rejected" and st["rejected"] == 1
    assert st["completed"] == 120 and st["submitted"] == 120
    assert st["batches"] < 120  # requests were batched
    assert srv.stats()["completed"] == 120  # final counters survive close
    for r in reqs:
        assert r.status == "done" and r.latency is not None and r.latency > 0
        alone = ccl.label(r.img, r.conn)
        torch.cuda.synchronize()
        assert torch.equal(alone, r.labels), r.rid
    for r in reqs[:10]:
        assert np.array_equal(r.labels.cpu().numpy(), _oracle(r.img, r.conn)[0])


def test_serve_waits_for_the_producing_stream(ccl):
    """A request submitted while its image is still being written on the
    current stream is labeled after that write (the ready stream)."""
    from paper_1606_05973_amd import serve
    srv = serve.Server(hbm_budget=128 << 20, n_streams=2, max_batch=4)
    side = torch.cuda.Stream()
    reqs, refs = [], []
    for i in range(6):
        src = inputs.bernoulli(400 + 50 * i, 500, 0.5, seed=40 + i, device=DEV)
        torch.cuda.synchronize()
        img = torch.zeros_like(src)
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            torch.cuda._sleep(2_000_000)  # keep the stream busy before the copy
            img.copy_(src)
            reqs.append(srv.submit(img, 8, level=0))
        refs.append(src)
    for r, src in zip(reqs, refs):
        assert r.wait()
        torch.cuda.synchronize()
        assert np.array_equal(r.labels.cpu().numpy(), _oracle(src, 8)[0])
    srv.close()


def test_serve_threshold_and_scan_options(ccl):
    from paper_1606_05973_amd import serve
    srv = serve.Server(hbm_budget=128 << 20, n_streams=2, max_batch=16)
    imgs = [inputs.gray(300 + 13 * i, 400, 2.0, seed=i, device=DEV) for i in range(8)]
    torch.cuda.synchronize()
    reqs = [srv.submit(im, 8 if i % 2 else 4, level=60 + 20 * i, scan=i % 2) for i, im in enumerate(imgs)]
    srv.drain()
    for i, (im, r) in enumerate(zip(imgs, reqs)):
        ref = oracle.label(im.cpu().numpy(), 8 if i % 2 else 4, level=60 + 20 * i)
        assert np.array_equal(r.labels.cpu().numpy(), ref)
    srv.close()


def test_captured_batch_call_replays(ccl):
    """ccl_label_batch captured into a graph (by torch, global capture mode)
    with several images: every replay labels the images' current content,
    with eager calls on the same stream between the replays."""
    specs = inputs.batch_specs(9, seed=41, max_side=500)
    imgs = [inputs.make(s_, device=DEV) for s_ in specs]
    conns = [8 if i % 3 else 4 for i in range(len(imgs))]
    outs = [torch.empty(tuple(im.shape), dtype=torch.int32, device=DEV) for im in imgs]
    k = torch.full((len(imgs),), -1, dtype=torch.int32, device=DEV)
    other = inputs.bernoulli(256, 300, 0.5, seed=8, device=DEV)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        ccl.reserve(ccl.batch_workspace_bytes([tuple(im.shape) for im in imgs], conns) + (1 << 20))
        ccl.label_batch(imgs, conns, outs=outs, num_components=k)   # eager warm-up on the same stream
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    say("case capture ccl_label_batch n=9")
    with torch.cuda.graph(g, stream=side):
        ccl.label_batch(imgs, conns, outs=outs, num_components=k)
    torch.cuda.synchronize()
    for rep in range(4):
        for i, (img, s_) in enumerate(zip(imgs, specs)):
            img.copy_(inputs.bernoulli(s_["H"], s_["W"], 0.25 + 0.15 * ((rep + i) % 4), seed=rep * 31 + i,
                                       device=DEV))
        k.fill_(-1)
        with torch.cuda.stream(side):
            eager = ccl.label(other, 8)      # same stream, same workspace, between replays
        torch.cuda.synchronize()
        say(f"case captured replay {rep}")
        g.replay()
        torch.cuda.synchronize()
        for i, img in enumerate(imgs):
            ref, kref = _oracle(img, conns[i])
            assert np.array_equal(outs[i].cpu().numpy(), ref), (rep, i)
            assert int(k[i].item()) == kref, (rep, i)
        assert np.array_equal(eager.cpu().numpy(), _oracle(other, 8)[0])
    del g
    torch.cuda.synchronize()


@pytest.mark.parametrize("slack", [0, -1])
def test_serve_admission_is_exact(ccl, slack):
    """A slot holding exactly the workspace of five mixed images (row pairs,
    single rows, gray levels: three launch groups) takes all five as one
    batch; one byte less and the fifth waits for the next batch."""
    from paper_1606_05973_amd import serve
    imgs = [inputs.bernoulli(300 + 40 * i, 700 - 30 * i, 0.5, seed=50 + i, device=DEV) for i in range(5)]
    conns = [8, 4, 8, 8, 4]
    scans = [0, 0, 1, 0, 0]
    grays = [False, False, False, True, False]
    need = ccl.batch_workspace_bytes([tuple(im.shape) for im in imgs], conns, 0, scans, grays)
    srv = serve.Server(hbm_budget=need + slack, n_streams=1, max_batch=16)
    blocker = torch.zeros((64, 64), dtype=torch.uint8, device=DEV)
    gate = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(gate):
        torch.cuda._sleep(500_000_000)   # the first batch waits on this stream (a fraction of a second)
        first = srv.submit(blocker, 8)
    time.sleep(0.005)                    # the scheduler has launched the blocker alone
    reqs = [srv.submit(im, c, scan=sc, gray=g) for im, c, sc, g in zip(imgs, conns, scans, grays)]
    srv.drain()
    st = srv.stats()
    srv.close()
    assert first.done
    assert st["batches"] == (2 if slack == 0 else 3), st
    for im, c, g, r in zip(imgs, conns, grays, reqs):
        host = im.cpu().numpy()
        ref = oracle.gray(host, c)[0] if g else oracle.cclremsp(host, c)[0]
        assert np.array_equal(r.labels.cpu().numpy(), ref)
