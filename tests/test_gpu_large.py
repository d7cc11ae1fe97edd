"""Maximum-size parity: an image whose guide and output hold more than 2^31
elements (64-bit offsets in every kernel), checked on sampled pixels and LR
cells against the oracle run on crops.

A pixel's result depends only on its window, so the oracle runs on the crop
of the LR cells within r of the pixel's cell (and their HR blocks); window
codes are relative to the pixel's cell, so the GPU's code is valid in the
crop unchanged.  A cell's gradient depends on the pixels whose window
reaches it, so the backward check crops the blocks within r of the cell."""
import numpy as np
import pytest
import torch

import oracle as O
import synth
from tests.gpu_util import host, log_case, need_gpu
from tests.parity import check_search

pytestmark = pytest.mark.gpu

H, W, S, K = 20000, 36000, 8, 3


def _glu():
    need_gpu()
    import paper_2307_09582_amd as glu

    return glu


def _crop_bounds(q, n_lr, n_hr, r):
    c0, c1 = max(0, q - r), min(n_lr, q + r + 1)
    return c0, c1, c0 * S, min(n_hr, c1 * S)


def test_search_apply_backward_beyond_2_31_elements():
    glu = _glu()
    log_case(test="large", H=H, W=W)
    assert H * W * 3 > 2**31
    dev = torch.device("cuda")
    base = torch.from_numpy(synth.voronoi(1000, 1200, n_cells=120, n_dots=40, dot_px=(1, 3), seed=31)).to(dev)
    I = base.repeat(H // 1000 + 1, W // 1200 + 1, 1)[:H, :W].contiguous()
    g = torch.Generator(device=dev)
    g.manual_seed(32)
    I.add_(0.01 * torch.randn(I.shape, generator=g, device=dev)).clamp_(0.0, 1.0)
    L = glu.downsample(I, S, "point")
    h, w = L.shape[:2]
    T = torch.rand((h, w, 3), generator=g, device=dev)
    out, th, err = glu.search_apply(I, L, T, S, K, 1e-3, "exhaustive", return_err=True)
    torch.cuda.synchronize()
    rng = np.random.default_rng(33)
    ys = np.concatenate([rng.integers(0, H, 400), [0, H - 1, H - 1, 0, H // 2], np.full(20, H - 1)])
    xs = np.concatenate([rng.integers(0, W, 400), [0, W - 1, 0, W - 1, W - 1], rng.integers(0, W, 20)])
    Lh = host(L)
    Th = host(T)
    r = K // 2
    for y, x in zip(ys.tolist(), xs.tolist()):
        cy0, cy1, y0, y1 = _crop_bounds(y // S, h, H, r)
        cx0, cx1, x0, x1 = _crop_bounds(x // S, w, W, r)
        Ic = host(I[y0:y1, x0:x1])
        Hc, Wc = Ic.shape[:2]
        code = np.zeros((Hc, Wc), np.int16)
        alpha = np.zeros((Hc, Wc), np.float32)
        e = np.zeros((Hc, Wc), np.float32)
        That = np.zeros((Hc, Wc, 3), np.float32)
        code[y - y0, x - x0] = int(th.code[y, x])
        alpha[y - y0, x - x0] = float(th.alpha[y, x])
        e[y - y0, x - x0] = float(err[y, x])
        That[y - y0, x - x0] = host(out[y, x])
        p = np.array([(y - y0) * Wc + (x - x0)])
        check_search(Ic, Lh[cy0:cy1, cx0:cx1], S, K, 1e-3, "exhaustive", code, alpha, err=e, pixels=p,
                     T_low=Th[cy0:cy1, cx0:cx1], T_hat=That)
    del out, err
    # backward: dalpha at the sampled pixels, grad_T_low at sampled cells,
    # each against the oracle's gradient of Eq. 1 on a crop
    G = torch.randn(I.shape, generator=g, device=dev)
    gT, ga = glu.apply_backward(th, T, G, S, K)
    torch.cuda.synchronize()

    def crop_backward(y0, y1, x0, x1, ly0, ly1, lx0, lx1, Gc):
        """Oracle gradients of Eq. 1 for the HR pixels [y0, y1) x [x0, x1)
        with LR indices relative to the LR crop [ly0, ly1) x [lx0, lx1)."""
        code = host(th.code[y0:y1, x0:x1]).astype(np.int64) & 0xFFFF
        al = host(th.alpha[y0:y1, x0:x1]).astype(np.float64)
        yy, xx = np.mgrid[y0:y1, x0:x1]
        o_a, o_b = np.divmod(code, K * K)
        lw = lx1 - lx0
        a = (yy // S + o_a // K - r - ly0) * lw + (xx // S + o_a % K - r - lx0)
        b = (yy // S + o_b // K - r - ly0) * lw + (xx // S + o_b % K - r - lx0)
        return O.apply_backward(a, b, al, Th[ly0:ly1, lx0:lx1], Gc)

    for y, x in zip(ys[:100].tolist(), xs[:100].tolist()):
        ly0, ly1, _, _ = _crop_bounds(y // S, h, H, r)
        lx0, lx1, _, _ = _crop_bounds(x // S, w, W, r)
        d_alpha, _ = crop_backward(y, y + 1, x, x + 1, ly0, ly1, lx0, lx1, host(G[y : y + 1, x : x + 1]))
        ref = float(d_alpha[0, 0])
        assert abs(float(ga[y, x]) - ref) <= 1e-5 * (1 + abs(ref))
    cells = [(0, 0), (h - 1, w - 1), (h // 2, w // 3), (h - 1, 0), (0, w - 1)]
    cells += [(int(rng.integers(0, h)), int(rng.integers(0, w))) for _ in range(25)]
    for qy, qx in cells:
        # pixels that can reach (qy, qx): the blocks within r of it, whose
        # windows lie within 2 r of it
        _, _, y0, y1 = _crop_bounds(qy, h, H, r)
        _, _, x0, x1 = _crop_bounds(qx, w, W, r)
        ly0, ly1, _, _ = _crop_bounds(qy, h, H, 2 * r)
        lx0, lx1, _, _ = _crop_bounds(qx, w, W, 2 * r)
        Gc = host(G[y0:y1, x0:x1]).astype(np.float64)
        _, dT = crop_backward(y0, y1, x0, x1, ly0, ly1, lx0, lx1, Gc)
        _, mass = crop_backward(y0, y1, x0, x1, ly0, ly1, lx0, lx1, np.abs(Gc))
        ref = dT[qy - ly0, qx - lx0]
        m = mass[qy - ly0, qx - lx0]
        got = host(gT[qy, qx]).astype(np.float64)
        assert np.all(np.abs(got - ref) <= 1e-5 * m + 1e-12), (qy, qx, got, ref)
