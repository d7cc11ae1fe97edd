"""GPU parity of the target-free overlap schedule (paper_2307_09582_amd.video).

The search reads the guide only (Sec. 3.1), so a video pipeline runs the
search of frame t on one stream while the LR operator computes frame t's
target on another (the paper's video use, Sec. 5.5).  Four float16 frames of
540 x 960 (x8) go through the overlapped schedule with a fixed LR operator:
every frame's LR guide equals the oracle's regular-grid downsample, Theta and
T_hat pass the per-pixel protocol against the oracle, and the outputs are
bitwise those of the one-stream schedule and of replays of a captured graph.
"""
import numpy as np
import pytest
import torch

import oracle as O
import synth
from tests.gpu_util import host, log_case, need_gpu
from tests.parity import check_search

pytestmark = pytest.mark.gpu

H, W, S, K, NF = 540, 960, 8, 3, 4
_M = {}


def _lr_op(c):
    """Fixed LR operator: the colour matrix, then gamma 0.8, in float32,
    stored as float16 (the matrix is uploaded once, outside any capture)."""
    m = _M.get(c.device)
    if m is None:
        m = _M[c.device] = torch.tensor(np.array(synth.COLOR_MATRIX, dtype=np.float32), device=c.device)
    return (torch.clamp(c.float() @ m.T, min=0.0) ** 0.8).half().contiguous()


def _frames():
    scene = synth.make_scene(H, W, 63, 25, (1, 3), seed=12, canvas_extra=3 * NF)
    return [scene.frame(t, sigma=0.01, dtype=np.float16) for t in range(NF)]


@pytest.mark.parametrize("mode", ["exhaustive", "fast"])
def test_overlapped_schedule_against_oracle(mode):
    need_gpu()
    from paper_2307_09582_amd import video

    log_case(test="overlap", mode=mode, H=H, W=W, frames=NF)
    frames_h = _frames()
    frames = [torch.from_numpy(f).cuda() for f in frames_h]
    side = torch.cuda.Stream()  # default priority
    with torch.no_grad():
        ref = video.sequential(frames, _lr_op, S, K, 1e-3, mode)
        ovl = video.overlapped(frames, _lr_op, side, S, K, 1e-3, mode)
        torch.cuda.synchronize()
        for t in range(NF):
            assert torch.equal(ovl.outs[t], ref.outs[t]), t
            assert torch.equal(ovl.thetas[t].code, ref.thetas[t].code)
            assert torch.equal(ovl.thetas[t].alpha, ref.thetas[t].alpha)
        for t in range(NF):
            L = O.downsample_point(frames_h[t], S)
            assert np.array_equal(host(ovl.lows[t]), L)
            rep = check_search(frames_h[t], L, S, K, 1e-3, mode, host(ovl.thetas[t].code), host(ovl.thetas[t].alpha),
                               T_low=host(ovl.targets[t]), T_hat=host(ovl.outs[t]), out_dtype=np.float16)
            print("frame", t, dict(rep), flush=True)

        # the same schedule captured as one graph (the side stream joins the
        # capture through its events), replayed with eager work in between
        bufs = video.VideoBuffers(frames, S)
        s0 = torch.cuda.Stream()
        s0.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s0):
            video.overlapped(frames, _lr_op, side, S, K, 1e-3, mode, bufs=bufs)
        torch.cuda.current_stream().wait_stream(s0)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            video.overlapped(frames, _lr_op, side, S, K, 1e-3, mode, bufs=bufs)
        for rep_i in range(3):
            for o in bufs.outs:
                o.zero_()
            g.replay()
            torch.cuda.synchronize()
            for t in range(NF):
                assert torch.equal(bufs.outs[t], ref.outs[t]), (rep_i, t)
            _lr_op(ref.lows[0]).float().sum().item()
        del g


def test_one_frame_forms_agree():
    """The latency forms (search submitted before the operator, or one
    stream) give bitwise the same frame."""
    need_gpu()
    from paper_2307_09582_amd import video

    frames = [torch.from_numpy(f).cuda() for f in _frames()[:1]]
    side = torch.cuda.Stream()
    with torch.no_grad():
        a = video.one_frame_sequential(frames[0], _lr_op, S, K, 1e-3, "exhaustive", video.VideoBuffers(frames, S))
        b = video.one_frame_overlapped(frames[0], _lr_op, side, S, K, 1e-3, "exhaustive", video.VideoBuffers(frames, S))
        torch.cuda.synchronize()
        assert torch.equal(a.outs[0], b.outs[0])
        assert torch.equal(a.thetas[0].code, b.thetas[0].code)
