"""GPU parity of the gradient-driven joint downsampling (glu_joint_downsample_grad)
against the float64 oracle, replayed step by step."""
import numpy as np
import pytest
import torch

import oracle as O
import synth
from tests.gpu_util import dev, host, log_case, need_gpu
from tests.parity import check_search, decode_codes

pytestmark = pytest.mark.gpu

SNAP_TIE = 1e-5  # Euclidean colour distance


def _glu():
    need_gpu()
    import paper_2307_09582_amd as glu

    return glu


def _blocks(I, s):
    H, W = I.shape[:2]
    h, w = H // s, W // s
    return I.reshape(h, s, w, s, 3).transpose(0, 2, 1, 3, 4).reshape(h * w, s * s, 3)


def _check_step(I, L_prev, th_prev, L_new, s, k, eta):
    """The GPU step from L_prev (with the GPU's Theta for it) moved every cell to
    a pixel of its block whose distance to the oracle's Z = L - eta D is within
    SNAP_TIE of the least."""
    H, W = I.shape[:2]
    h, w = H // s, W // s
    pix = np.arange(H * W, dtype=np.int64)
    a, b, ok = decode_codes(host(th_prev.code), H, W, s, k, pix)
    assert ok.all()
    alpha = host(th_prev.alpha).astype(np.float64).reshape(-1)
    D, _ = O.self_upsampling_gradient(I, L_prev, a, b, alpha)
    Z = (np.asarray(L_prev, np.float64) - eta * D).reshape(h * w, 3)
    blk = _blocks(np.asarray(I, np.float64), s)
    dmin = np.sqrt(((blk - Z[:, None, :]) ** 2).sum(-1).min(axis=1))
    Ln = np.asarray(L_new, np.float64).reshape(h * w, 3)
    dg = np.sqrt(((Ln - Z) ** 2).sum(-1))
    gap = dg - dmin
    assert gap.max() <= SNAP_TIE, "snap is not the nearest pixel (gap %.3g at cell %d)" % (gap.max(), gap.argmax())
    member = np.any(np.all(blk == Ln[:, None, :], axis=-1), axis=1)
    assert member.all(), "I_low pixel that is not a copy of an HR pixel of its block"
    return int((gap > 0).sum())


@pytest.mark.parametrize("mode", ["exhaustive", "fast"])
def test_step_replay(mode):
    glu = _glu()
    log_case(test="jdgrad_step_replay", mode=mode)
    s, k, eta = 8, 3, 0.01
    I = synth.voronoi(96, 120, n_cells=20, n_dots=10, dot_px=(1, 3), seed=7)
    dI = dev(I)
    L = O.downsample_point(I, s).astype(np.float32)
    th, _ = glu.search(dI, dev(L), s, k, 1e-3, mode, return_err=True)
    for t in range(3):
        Lg, thg, Eg, sums, best = glu.joint_downsample_grad(dI, dev(L), s, k, 1e-3, mode, eta, 1, keep_best=False)
        assert best == 1
        Lgh = host(Lg)
        _check_step(I, L, th, Lgh, s, k, eta)
        check_search(I, Lgh, s, k, 1e-3, mode, host(thg.code), host(thg.alpha), err=host(Eg))
        e64 = float(host(Eg).astype(np.float64).sum())
        assert abs(sums[1] - e64) <= 1e-9 * max(1.0, e64)
        L, th = Lgh, thg


def test_full_run_keeps_the_best_and_eta_zero_is_fixed():
    glu = _glu()
    log_case(test="jdgrad_full_run")
    s, k = 8, 3
    I = synth.voronoi(128, 160, n_cells=30, n_dots=12, dot_px=(1, 3), seed=9)
    dI = dev(I)
    L0 = O.downsample_point(I, s).astype(np.float32)
    Lg, thg, Eg, sums, best = glu.joint_downsample_grad(dI, dev(L0), s, k, eta=0.05, n_steps=5, keep_best=True)
    assert len(sums) == 6 and best == int(np.argmin(sums))
    e64 = float(host(Eg).astype(np.float64).sum())
    assert abs(e64 - min(sums)) <= 1e-9 * max(1.0, e64)
    Lgh = host(Lg)
    check_search(I, Lgh, s, k, 1e-3, "exhaustive", host(thg.code), host(thg.alpha), err=host(Eg))
    blk = _blocks(np.asarray(I, np.float64), s)
    assert np.any(np.all(blk == Lgh.reshape(-1, 3)[:, None, :].astype(np.float64), axis=-1), axis=1).all()
    # the last I_low when not keeping the best, and eta = 0 leaves I_low as it is
    Ll, _, _, sums2, best2 = glu.joint_downsample_grad(dI, dev(L0), s, k, eta=0.05, n_steps=5, keep_best=False)
    assert best2 == 5 and sums2 == sums
    L0g, _, _, sums0, _ = glu.joint_downsample_grad(dI, dev(L0), s, k, eta=0.0, n_steps=2, keep_best=False)
    assert np.array_equal(host(L0g), L0) and sums0[0] == sums0[1] == sums0[2]
    # deterministic
    Lg2, _, _, sums3, _ = glu.joint_downsample_grad(dI, dev(L0), s, k, eta=0.05, n_steps=5, keep_best=True)
    assert torch.equal(Lg2, Lg) and sums3 == sums


def test_2048_x8_five_steps():
    """The joint-downsampling workload size (2048 x 2048, x8, 5 steps): the sum
    of E does not increase, and the final Theta and E pass the parity protocol
    on sampled pixels."""
    glu = _glu()
    log_case(test="jdgrad_2048")
    s, k = 8, 3
    I = synth.voronoi(2048, 2048, n_cells=512, n_dots=200, dot_px=(1, 3), seed=2)
    dI = dev(I)
    L0 = O.downsample_point(I, s).astype(np.float32)
    Lg, thg, Eg, sums, best = glu.joint_downsample_grad(dI, dev(L0), s, k, eta=0.01, n_steps=5, keep_best=True)
    assert min(sums) <= sums[0]
    print("sums", sums, "best", best)
    rng = np.random.default_rng(0)
    pix = rng.choice(2048 * 2048, 20000, replace=False)
    check_search(I, host(Lg), s, k, 1e-3, "exhaustive", host(thg.code), host(thg.alpha), err=host(Eg), pixels=pix)
