"""GPU parity of glu_joint_downsample (Algorithm 2) against the oracle.

Decision replay: the oracle runs Algorithm 2 and, at every decision where it
disagrees with the GPU's decision log, requires a near-tie (arg-max E gap
<= 1e-6; |e1 - e0| <= 1e-6 |A| for the accept test) and then adopts the
GPU's choice.  After that the optimised I_low must match bitwise (it holds
copies of HR pixels), the per-round counts must be equal, and Theta / E must
pass the per-pixel search protocol against the final I_low.
"""
import numpy as np
import pytest

import oracle as O
import synth
from tests.gpu_util import dev, host, log_case, need_gpu
from tests.parity import check_search

pytestmark = pytest.mark.gpu


def _glu():
    need_gpu()
    import paper_2307_09582_amd as glu

    return glu


class Replay:
    def __init__(self, gpu_log):
        self.log = gpu_log
        self.cursor = 0
        self.replays = 0

    def __call__(self, kind, payload, default):
        if kind == "membership":
            return default
        g = self.log[self.cursor]
        if kind == "argmax":
            q, members, Em = payload
            gp = dict(g["q_pstar"])[q]
            if gp != default:
                idx = list(members).index(gp)
                gap = float(Em.max() - Em[idx])
                assert gap <= 1e-6, "arg-max mismatch at q=%d (gap %.3g)" % (q, gap)
                self.replays += 1
            return gp
        if kind == "accept":
            e0, e1, na = payload
            self.cursor += 1
            if g["accepted"] != default:
                assert abs(e1 - e0) <= 1e-6 * na, "accept mismatch: e0=%.9g e1=%.9g |A|=%d" % (e0, e1, na)
                self.replays += 1
            return g["accepted"]
        raise AssertionError(kind)


def _check(glu, I, L0, s, k, mode, tau, n_iter, check_all_pixels=True):
    I = np.ascontiguousarray(I.astype(np.float32))
    L0 = np.ascontiguousarray(L0.astype(np.float32))
    Lg, th, err, stats, log = glu.joint_downsample(dev(I), dev(L0), s, k, 1e-3, mode, tau, n_iter)
    Lg = host(Lg)
    assert not stats.get("log_truncated")
    rp = Replay(log)
    ref = O.joint_downsample(I, L0, s, k, 1e-3, mode, tau, n_iter, decide=rp)
    assert rp.cursor == len(log), (rp.cursor, len(log))
    assert ref.rounds_run == stats["rounds_run"]
    assert ref.n_large == stats["n_large"] and ref.n_components == stats["n_components"]
    assert ref.n_accepted == stats["n_accepted"]
    for d, g in zip(ref.log, log):
        assert d.first_pixel == g["first_pixel"] and d.round == g["round"]
        assert [q for q, _ in d.q_pstar] == [q for q, _ in g["q_pstar"]]
        assert abs(d.e0 - g["e0"]) <= 1e-6 * max(1.0, d.e0) + 1e-5 and abs(d.e1 - g["e1"]) <= 1e-6 * max(1.0, d.e1) + 1e-5
    # the optimised LR guide holds copies of HR pixels: bitwise equal
    assert np.array_equal(Lg, ref.L.astype(np.float32))
    n = I.shape[0] * I.shape[1]
    assert abs(stats["err_sum_initial"] - ref.err_sum_initial) <= 1e-6 * n
    assert abs(stats["err_sum_final"] - ref.err_sum_final) <= 1e-6 * n
    pix = None if check_all_pixels else np.random.default_rng(0).choice(n, 50000, replace=False)
    check_search(I, Lg, s, k, 1e-3, mode, host(th.code), host(th.alpha), err=host(err), pixels=pix)
    return stats, log, rp


def _dot_image(H=64, W=64, dot=(17, 41), size=2):
    I = np.empty((H, W, 3), np.float32)
    I[:] = (0.4, 0.5, 0.6)
    I[dot[0] : dot[0] + size, dot[1] : dot[1] + size] = (0.95, 0.1, 0.1)
    return I


@pytest.mark.parametrize("mode", ["exhaustive", "fast"])
def test_dot_recovery(mode):
    glu = _glu()
    I = _dot_image()
    L0 = O.downsample_point(I, 8)
    stats, log, _ = _check(glu, I, L0, 8, 3, mode, O.TAU, 3)
    assert stats["n_components"][0] == 1 and stats["n_accepted"][0] == 1 and stats["rounds_run"] == 1


def test_rollback():
    glu = _glu()
    I = np.empty((24, 24, 3), np.float32)
    I[:] = (0.6, 0.6, 0.6)
    I[8:16, 8:16] = (0.2, 0.2, 0.2)
    I[9:11, 9:11] = (0.9, 0.1, 0.1)
    L0 = O.downsample_point(I, 8)
    stats, log, _ = _check(glu, I, L0, 8, 3, "exhaustive", O.TAU, 1)
    assert len(log) == 1 and not log[0]["accepted"] and log[0]["e1"] > log[0]["e0"]


# n_dots: dots of 1-3 px, 32 px apart; at s = 3 regular-grid sampling
# already catches most of them, so that case takes 12 dots to keep several
# trials (3 components in round 1)
@pytest.mark.parametrize("mode,H,W,s,k,n_dots", [("exhaustive", 256, 320, 8, 3, 20), ("fast", 256, 320, 8, 3, 20),
                                                 ("exhaustive", 203, 157, 4, 3, 7), ("exhaustive", 160, 160, 8, 5, 6),
                                                 ("exhaustive", 97, 131, 3, 3, 12)])
def test_voronoi(mode, H, W, s, k, n_dots):
    glu = _glu()
    log_case(test="joint_voronoi", mode=mode, H=H, W=W, s=s, k=k)
    I = synth.voronoi(H, W, n_cells=max(8, H * W // 2000), n_dots=n_dots, dot_px=(1, 3), seed=H + W)
    L0 = O.downsample_point(I, s)
    stats, log, rp = _check(glu, I, L0, s, k, mode, O.TAU, 3)
    assert stats["rounds_run"] >= 1 and len(log) >= 3
    print(stats, "replays", rp.replays)


def test_no_large_error_and_zero_iterations():
    glu = _glu()
    rng = np.random.default_rng(3)
    L = rng.uniform(0, 1, (9, 11, 3)).astype(np.float32)
    I = np.ascontiguousarray(np.repeat(np.repeat(L, 4, 0), 4, 1))
    Lg, th, err, stats, log = glu.joint_downsample(dev(I), dev(L), 4, 3)
    assert stats["rounds_run"] == 0 and log == []
    assert np.array_equal(host(Lg), L)
    I2 = synth.voronoi(64, 64, n_cells=6, n_dots=6, seed=4)
    L2 = O.downsample_point(I2, 8)
    Lg2, th2, err2, stats2, log2 = glu.joint_downsample(dev(I2), dev(L2), 8, 3, max_iter=0)
    assert stats2["rounds_run"] == 0 and np.array_equal(host(Lg2), L2)
    th3, e3 = glu.search(dev(I2), dev(L2), 8, 3, return_err=True)
    assert np.array_equal(host(th2.code), host(th3.code)) and np.array_equal(host(err2), host(e3))


def test_determinism():
    glu = _glu()
    I = synth.voronoi(192, 256, n_cells=30, n_dots=20, dot_px=(1, 3), seed=8)
    L0 = O.downsample_point(I, 8)
    a = glu.joint_downsample(dev(I), dev(L0), 8, 3)
    b = glu.joint_downsample(dev(I), dev(L0), 8, 3)
    assert np.array_equal(host(a[0]), host(b[0]))
    assert np.array_equal(host(a[1].code), host(b[1].code)) and np.array_equal(host(a[2]), host(b[2]))
    assert a[3] == b[3] and a[4] == b[4]


def test_joint_2048_x8_five_rounds():
    """The 2048 x 2048 x8 workload with five rounds (512 cells, 200 dots of
    1-3 px), checked by decision replay; Theta / E on 50000 sampled pixels."""
    glu = _glu()
    log_case(test="joint_2048_x8")
    I = synth.voronoi(2048, 2048, n_cells=512, n_dots=200, dot_px=(1, 3), seed=2)
    L0 = O.downsample_point(I, 8)
    stats, log, rp = _check(glu, I, L0, 8, 3, "exhaustive", O.TAU, 5, check_all_pixels=False)
    print(stats, "replays", rp.replays)
    assert stats["err_sum_final"] <= stats["err_sum_initial"]


def test_giant_component_box_walk():
    """One component covering the whole image (tau = 0 on noise): its 16384
    affected LR cells exceed the trial's LDS list, so the trial walks the
    component's bounding box instead; decisions, I_low and Theta as the
    oracle's."""
    glu = _glu()
    log_case(test="joint_giant_component")
    rng = np.random.default_rng(17)
    I = rng.uniform(0, 1, (256, 256, 3)).astype(np.float32)
    L0 = O.downsample_point(I, 2)
    stats, log, _ = _check(glu, I, L0, 2, 3, "exhaustive", 0.0, 1)
    assert stats["n_components"][0] == 1 and len(log) == 1


# Theta and E returned by Algorithm 2 are maintained by the trials (a kept
# trial commits its affected set's re-search); they must be bitwise those of
# a full search against the returned I_low.  Cases with kept trials in both
# modes, 3 x 3 and 5 x 5 windows, and components at the image border.
@pytest.mark.parametrize("mode,H,W,s,k", [("exhaustive", 256, 320, 8, 3), ("fast", 256, 320, 8, 3),
                                          ("exhaustive", 203, 157, 4, 3), ("fast", 203, 157, 3, 3),
                                          ("exhaustive", 160, 168, 8, 5), ("fast", 150, 170, 6, 5)])
def test_returned_theta_is_a_full_search(mode, H, W, s, k):
    glu = _glu()
    log_case(test="joint_theta_is_full_search", mode=mode, H=H, W=W, s=s, k=k)
    I = synth.voronoi(H, W, n_cells=max(8, H * W // 2000), n_dots=24, dot_px=(1, 3), seed=H * 7 + W)
    L0 = O.downsample_point(I, s)
    dI = dev(np.ascontiguousarray(I.astype(np.float32)))
    Lg, th, err, stats, log = glu.joint_downsample(dI, dev(np.ascontiguousarray(L0.astype(np.float32))), s, k,
                                                   1e-3, mode, O.TAU, 4)
    assert sum(stats["n_accepted"][: stats["rounds_run"]]) >= 1, stats
    th2, e2 = glu.search(dI, Lg, s, k, 1e-3, mode, return_err=True)
    assert np.array_equal(host(th.code), host(th2.code))
    assert np.array_equal(host(th.alpha), host(th2.alpha))
    assert np.array_equal(host(err), host(e2))
