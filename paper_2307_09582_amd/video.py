"""Frame schedules for video: the search overlapped with the LR operator.

The pair search reads the high-resolution guide and its downsampled copy
only, never the low-resolution target (Sec. 3.1), so in a video pipeline the
search of a frame can run while the LR operator f is still computing that
frame's target; only the apply step (Eq. 1) needs both.  The paper uses this
to run its GPU upsampler beside the LR operator for video (Sec. 5.5).

``overlapped`` issues, per frame t on the current stream: the regular-grid
downsample, the search of frame t, then the apply of frame t - 1, which
waits for that frame's target; the operator of frame t runs on ``side``
after the downsample.  ``sequential`` runs downsample, operator and the
fused search + apply of each frame on the current stream.  Both give
bitwise the same outputs (the fused pass and the two-kernel form agree
bitwise).  Streams keep the default priority.  Every kernel of the upsampler
is a HIP kernel of libglu; ``lr_op`` is the caller's operator (any torch
code producing the frame's target from its LR guide).
"""
from __future__ import annotations

import torch

from . import glu as _glu


class VideoBuffers:
    """Per-frame LR guides, targets, Theta and outputs of a schedule, sized
    for ``frames`` (a list of (H, W, 3) GPU tensors of one shape and dtype)
    and an operator returning ``channels`` target channels."""

    def __init__(self, frames, s: int, channels: int = 3):
        if not frames:
            raise ValueError("no frames")
        H, W = frames[0].shape[:2]
        dev, dt = frames[0].device, frames[0].dtype
        h, w = _glu.lr_shape(H, W, s)
        self.lows = [torch.empty((h, w, 3), dtype=dt, device=dev) for _ in frames]
        self.targets = [None] * len(frames)
        self.thetas = [_glu.empty_theta(H, W, dev) for _ in frames]
        self.outs = [torch.empty((H, W, channels), dtype=dt, device=dev) for _ in frames]


def _down(frame, low, s):
    _glu.downsample(frame, s, "point", out=low)


def _keep_for(t: torch.Tensor, stream: torch.cuda.Stream):
    """A tensor made on another stream is read on ``stream``: its memory is
    not reused before that stream's work is done (a graph capture keeps its
    own pool, so nothing is needed there)."""
    if not torch.cuda.is_current_stream_capturing():
        t.record_stream(stream)


def sequential(frames, lr_op, s, k=3, eps=_glu.EPS, mode="exhaustive", bufs: VideoBuffers | None = None):
    """Downsample, operator and fused search + apply per frame, one stream."""
    bufs = bufs or VideoBuffers(frames, s)
    for t, f in enumerate(frames):
        _down(f, bufs.lows[t], s)
        bufs.targets[t] = lr_op(bufs.lows[t])
        _glu.search_apply(f, bufs.lows[t], bufs.targets[t], s, k, eps, mode, theta=bufs.thetas[t], out=bufs.outs[t])
    return bufs


def overlapped(frames, lr_op, side: torch.cuda.Stream, s, k=3, eps=_glu.EPS, mode="exhaustive",
               bufs: VideoBuffers | None = None):
    """The search of frame t on the current stream while the operator of
    frame t runs on ``side``; the apply of frame t - 1 follows the search of
    frame t.  Returns the buffers (outputs in ``bufs.outs``)."""
    bufs = bufs or VideoBuffers(frames, s)
    main = torch.cuda.current_stream()
    ready = [torch.cuda.Event() for _ in frames]
    n = len(frames)
    for t, f in enumerate(frames):
        _down(f, bufs.lows[t], s)
        low_done = torch.cuda.Event()
        low_done.record(main)
        side.wait_event(low_done)
        with torch.cuda.stream(side):
            bufs.targets[t] = lr_op(bufs.lows[t])
            ready[t].record(side)
        _keep_for(bufs.targets[t], main)
        _glu.search(f, bufs.lows[t], s, k, eps, mode, theta=bufs.thetas[t])
        if t > 0:
            main.wait_event(ready[t - 1])
            _glu.apply(bufs.thetas[t - 1], bufs.targets[t - 1], s, k, out=bufs.outs[t - 1])
    main.wait_event(ready[n - 1])
    _glu.apply(bufs.thetas[n - 1], bufs.targets[n - 1], s, k, out=bufs.outs[n - 1])
    return bufs


def one_frame_overlapped(frame, lr_op, side: torch.cuda.Stream, s, k, eps, mode, bufs: VideoBuffers, t: int = 0):
    """One frame with the search submitted before the operator (the
    latency form): downsample, search, operator on ``side``, then apply."""
    main = torch.cuda.current_stream()
    _down(frame, bufs.lows[t], s)
    low_done, ready = torch.cuda.Event(), torch.cuda.Event()
    low_done.record(main)
    _glu.search(frame, bufs.lows[t], s, k, eps, mode, theta=bufs.thetas[t])
    side.wait_event(low_done)
    with torch.cuda.stream(side):
        bufs.targets[t] = lr_op(bufs.lows[t])
        ready.record(side)
    _keep_for(bufs.targets[t], main)
    main.wait_event(ready)
    _glu.apply(bufs.thetas[t], bufs.targets[t], s, k, out=bufs.outs[t])
    return bufs


def one_frame_sequential(frame, lr_op, s, k, eps, mode, bufs: VideoBuffers, t: int = 0):
    """One frame on one stream: downsample, operator, fused search + apply."""
    _down(frame, bufs.lows[t], s)
    bufs.targets[t] = lr_op(bufs.lows[t])
    _glu.search_apply(frame, bufs.lows[t], bufs.targets[t], s, k, eps, mode, theta=bufs.thetas[t], out=bufs.outs[t])
    return bufs
