"""The batched workloads at full size, in the launches the benchmark times,
against the oracle (Eq. 3-5 for the search, Eq. 1 for T_hat).

* 60 frames of 3840 x 2160 float16 video, x8, 3 x 3, one launch of one
  kernel variant replayed from a captured graph, no Theta stored.
* 64 float32 images of uneven size (720 x 480 .. 6000 x 4000), s in
  {4, 8, 16}, k in {3, 5}, tiles autotuned per (s, k), one launch per
  variant group, no Theta stored.

Each plan runs a second time with Theta stored; T_hat must be bitwise the
same, and the stored Theta and that T_hat are checked against the oracle:
every pixel of some images, sampled pixels of all the others.  The oracle's
search runs in a pool of host processes (tests/parity.py)."""
import numpy as np
import pytest
import torch

import oracle as O
import synth
from tests.gpu_util import host, log_case, need_gpu
from tests.parity import check_search

pytestmark = pytest.mark.gpu

EPS = 1e-3
VIDEO_FULL = (0, 29, 59)  # frames checked on every pixel
VIDEO_SAMPLES = 20000  # pixels checked in each other frame
UNEVEN_SAMPLES = 5000


def _glu():
    need_gpu()
    import paper_2307_09582_amd as glu

    return glu


@pytest.fixture(scope="module")
def video():
    glu = _glu()
    canvas = torch.from_numpy(synth.scene_4k().canvas.astype(np.float32)).cuda()
    items = []
    for If in synth.video_frames_torch(canvas, 60, torch.float16):
        Il = glu.downsample(If, 8, "point")
        items.append(dict(I=If, I_low=Il, T_low=synth.lr_op_f1_torch(Il).half().contiguous(), s=8, k=3))
    del canvas
    yield items
    items.clear()
    torch.cuda.empty_cache()


@pytest.fixture(scope="module")
def uneven():
    glu = _glu()
    specs = synth.uneven_batch_specs(64, seed=4)
    uc = synth.UNEVEN_CANVAS
    big = synth.make_scene(uc["H"], uc["W"], uc["n_cells"], uc["n_dots"], uc["dot_px"], seed=uc["seed"])
    canvas = torch.from_numpy(big.canvas.astype(np.float32)).cuda()
    del big
    imgs, _ = synth.uneven_batch_torch(canvas, specs, torch.float32)
    del canvas
    items = []
    for Iu, sp in zip(imgs, specs):
        Il = glu.downsample(Iu, sp["s"], "point")
        items.append(dict(I=Iu, I_low=Il, T_low=synth.lr_op_f1_torch(Il).contiguous(), s=sp["s"], k=sp["k"]))
    del imgs
    yield items
    items.clear()
    torch.cuda.empty_cache()


def _run_twice(glu, items, mode, graph):
    """The benchmark's plan (no Theta), then the same items with Theta
    stored; returns the second set of items after checking that both wrote
    bitwise the same T_hat."""
    bench = [dict(it, T_hat=torch.empty_like(it["I"])) for it in items]
    plan = glu.BatchPlan(bench, mode=mode)
    if graph:
        g = plan.capture_graph()
        g.replay()
    else:
        plan.launch()
    torch.cuda.synchronize()
    chk = [dict(it, T_hat=torch.empty_like(it["I"]), theta=glu.empty_theta(*it["I"].shape[:2])) for it in items]
    plan2 = glu.BatchPlan(chk, mode=mode)
    plan2.launch()
    torch.cuda.synchronize()
    for i, (a, b) in enumerate(zip(bench, chk)):
        assert torch.equal(a["T_hat"], b["T_hat"]), "T_hat of item %d depends on storing Theta" % i
    if graph:
        del g
    plan.close()
    plan2.close()
    del bench
    return chk


def _check(pool, it, mode, pixels, out_dtype):
    I = host(it["I"])
    L = host(it["I_low"])
    s, k = it["s"], it["k"]
    assert np.array_equal(L, O.downsample_point(I, s))
    ref = pool.search(I, L, s, k, EPS, mode, pixels=pixels)
    return check_search(I, L, s, k, EPS, mode, host(it["theta"].code), host(it["theta"].alpha), pixels=pixels,
                        T_low=host(it["T_low"].float()), T_hat=host(it["T_hat"]), out_dtype=out_dtype, ref=ref)


@pytest.mark.parametrize("mode", ["exhaustive", "fast"])
def test_video_60x4k_f16_bench_launch(video, oracle_pool, mode):
    glu = _glu()
    log_case(test="video_60x4k_f16_bench_launch", mode=mode)
    chk = _run_twice(glu, video, mode, graph=True)
    H, W = 2160, 3840
    rng = np.random.default_rng(60)
    ties = checked = 0
    for t, it in enumerate(chk):
        pix = None if t in VIDEO_FULL else np.sort(rng.choice(H * W, VIDEO_SAMPLES, replace=False))
        rep = _check(oracle_pool, it, mode, pix, np.float16)
        ties += rep["near_ties"]
        checked += rep["n"]
        if t in VIDEO_FULL:
            print("frame", t, "every pixel:", dict(rep), flush=True)
    print(mode, "checked", checked, "pixels, near-ties", ties, flush=True)
    del chk
    torch.cuda.empty_cache()


@pytest.mark.parametrize("mode", ["exhaustive", "fast"])
def test_uneven_64_bench_launch(uneven, oracle_pool, mode):
    glu = _glu()
    log_case(test="uneven_64_bench_launch", mode=mode)
    seen = set()
    for it in uneven:
        if (it["s"], it["k"]) not in seen:
            seen.add((it["s"], it["k"]))
            glu.autotune(dict(it, T_hat=torch.empty_like(it["I"])), mode=mode)
    chk = _run_twice(glu, uneven, mode, graph=False)
    # every pixel of the smallest image of each (s, k) group
    full = {}
    for i, it in enumerate(chk):
        key = (it["s"], it["k"])
        n = it["I"].shape[0] * it["I"].shape[1]
        if key not in full or n < full[key][1]:
            full[key] = (i, n)
    full_idx = {i for i, _ in full.values()}
    assert len(full) == 6
    rng = np.random.default_rng(64)
    ties = checked = 0
    for i, it in enumerate(chk):
        n = it["I"].shape[0] * it["I"].shape[1]
        pix = None if i in full_idx else np.sort(rng.choice(n, UNEVEN_SAMPLES, replace=False))
        rep = _check(oracle_pool, it, mode, pix, np.float32)
        ties += rep["near_ties"]
        checked += rep["n"]
        if i in full_idx:
            print("image", i, tuple(it["I"].shape[:2]), "s", it["s"], "k", it["k"], "every pixel:", dict(rep),
                  flush=True)
    print(mode, "checked", checked, "pixels, near-ties", ties, flush=True)
    del chk
    torch.cuda.empty_cache()
