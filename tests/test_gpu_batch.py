"""Batched execution (one launch per kernel variant), hipGraph capture and the autotuner."""
import os

import numpy as np
import pytest
import torch

import oracle as O
import synth
from tests.gpu_util import dev, host, log_case, need_gpu
from tests.parity import check_search

pytestmark = pytest.mark.gpu


def _glu():
    need_gpu()
    import paper_2307_09582_amd as glu

    return glu


def _item(H, W, s, k, C, dtype, seed, with_theta=True):
    glu = _glu()
    I = synth.voronoi(H, W, n_cells=max(4, H * W // 3000), n_dots=max(2, H * W // 8000), dot_px=(1, 3), seed=seed)
    L = O.downsample_point(I, s)
    T = synth.lr_op_f1(L)[..., :C]
    tdt = torch.float16 if dtype == "f16" else torch.float32
    it = dict(I=dev(I).to(tdt), I_low=dev(L).to(tdt), T_low=dev(T.astype(np.float32)).to(tdt), s=s, k=k)
    it["T_hat"] = torch.empty((H, W, C), dtype=tdt, device="cuda")
    it["theta"] = glu.empty_theta(H, W) if with_theta else None
    return it


SPECS = [
    (128, 200, 8, 3, 3, "f32"),
    (97, 61, 4, 5, 1, "f32"),
    (64, 64, 16, 3, 3, "f16"),
    (45, 77, 3, 3, 3, "f32"),
    (200, 120, 8, 7, 2, "f32"),
    (33, 250, 2, 3, 3, "f16"),
    (1, 1, 1, 3, 1, "f32"),
    (260, 300, 4, 3, 3, "f32"),
    (90, 110, 6, 3, 3, "f32"),
    (52, 70, 10, 5, 2, "f16"),
    (64, 96, 8, 5, 3, "f32"),
]


@pytest.mark.parametrize("mode", ["exhaustive", "fast"])
def test_batch_equals_single_image(mode):
    glu = _glu()
    log_case(test="batch_equals_single", mode=mode)
    items = [_item(*sp, seed=i + 1, with_theta=(i % 3 != 1)) for i, sp in enumerate(SPECS)]
    plan = glu.BatchPlan(items, mode=mode)
    nt, ng = plan.info()
    assert nt > 0 and ng > 0
    plan.launch()
    torch.cuda.synchronize()
    for it in items:
        out, th = glu.search_apply(it["I"], it["I_low"], it["T_low"], it["s"], it["k"], mode=mode)
        assert torch.equal(out, it["T_hat"])
        if it["theta"] is not None:
            assert torch.equal(th.code, it["theta"].code) and torch.equal(th.alpha, it["theta"].alpha)
    # parity with the oracle on two items
    for it in (items[0], items[3]):
        I = host(it["I"].float())
        L = host(it["I_low"].float())
        T = host(it["T_low"].float())
        check_search(I, L, it["s"], it["k"], 1e-3, mode, host(it["theta"].code), host(it["theta"].alpha),
                     T_low=T, T_hat=host(it["T_hat"].float()))


def test_graph_capture_replays():
    glu = _glu()
    items = [_item(*sp, seed=10 + i) for i, sp in enumerate(SPECS[:5])]
    plan = glu.BatchPlan(items)
    plan.launch()
    torch.cuda.synchronize()
    ref = [it["T_hat"].clone() for it in items]
    refc = [it["theta"].code.clone() for it in items]
    g = plan.capture_graph()
    for rep in range(3):
        for it in items:  # eager work between replays
            it["T_hat"].zero_()
            it["theta"].code.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for it, r, rc in zip(items, ref, refc):
            assert torch.equal(it["T_hat"], r), rep
            assert torch.equal(it["theta"].code, rc), rep


def test_video_frames_fp16():
    """A short fp16 video of a translating scene in one launch (the frames of
    the 4K video workload, at 960 x 540)."""
    glu = _glu()
    scene = synth.make_scene(540, 960, 100, 40, (1, 3), seed=3, canvas_extra=30)
    items = []
    for t in range(8):
        I = scene.frame(t, sigma=0.01, dtype=np.float32)
        L = O.downsample_point(I, 8)
        T = synth.lr_op_f1(L).astype(np.float32)
        items.append(dict(I=dev(I).half(), I_low=dev(L).half(), T_low=dev(T).half(), s=8, k=3,
                          T_hat=torch.empty((540, 960, 3), dtype=torch.float16, device="cuda"),
                          theta=glu.empty_theta(540, 960)))
    plan = glu.BatchPlan(items)
    plan.launch()
    torch.cuda.synchronize()
    for t in (0, 7):
        it = items[t]
        check_search(host(it["I"].float()), host(it["I_low"].float()), 8, 3, 1e-3, "exhaustive",
                     host(it["theta"].code), host(it["theta"].alpha), T_low=host(it["T_low"].float()),
                     T_hat=host(it["T_hat"]), out_dtype=np.float16,
                     pixels=np.random.default_rng(t).choice(540 * 960, 20000, replace=False))


def test_autotune_and_cache_file(tmp_path):
    glu = _glu()
    it = _item(512, 640, 8, 3, 3, "f32", seed=31)
    v = glu.autotune(it)
    assert 0 <= v < 8
    path = str(tmp_path / "tune.json")
    glu.autotune_save(path)
    txt = open(path).read()
    assert '"variant": %d' % v in txt
    glu.autotune_load(path)
    # plans and single-image calls use the tuned tile; results stay correct
    plan = glu.BatchPlan([it])
    plan.launch()
    out, th = glu.search_apply(it["I"], it["I_low"], it["T_low"], 8, 3)
    assert torch.equal(out, it["T_hat"])
    check_search(host(it["I"]), host(it["I_low"]), 8, 3, 1e-3, "exhaustive", host(it["theta"].code),
                 host(it["theta"].alpha), T_low=host(it["T_low"]), T_hat=host(it["T_hat"]),
                 pixels=np.random.default_rng(1).choice(512 * 640, 20000, replace=False))


def test_uneven_batch_small():
    """Uneven sizes, factors {4, 8, 16} and windows {3, 5}, scaled down 8x."""
    glu = _glu()
    specs = synth.uneven_batch_specs(12, seed=4, wmin=90, wmax=750, hmin=60, hmax=500)
    items = []
    for sp in specs:
        items.append(_item(sp["H"], sp["W"], sp["s"], sp["k"], 3, "f32", seed=sp["seed"]))
    plan = glu.BatchPlan(items)
    plan.launch()
    torch.cuda.synchronize()
    for it in items[:4]:
        n = it["I"].shape[0] * it["I"].shape[1]
        check_search(host(it["I"]), host(it["I_low"]), it["s"], it["k"], 1e-3, "exhaustive", host(it["theta"].code),
                     host(it["theta"].alpha), T_low=host(it["T_low"]), T_hat=host(it["T_hat"]),
                     pixels=np.random.default_rng(2).choice(n, min(n, 10000), replace=False))


def test_empty_plan_and_validation():
    glu = _glu()
    plan = glu.BatchPlan([])
    plan.launch()
    it = _item(64, 64, 8, 3, 3, "f32", seed=1)
    bad = dict(it)
    bad["I_low"] = torch.empty((3, 3, 3), device="cuda")
    with pytest.raises(glu.GluError):
        glu.BatchPlan([it, bad])
