"""GPU parity of glu_apply_backward and the GluApply autograd function."""
import numpy as np
import pytest
import torch

import oracle as O
import synth
from tests.gpu_util import dev, host, log_case, need_gpu

pytestmark = pytest.mark.gpu


def _glu():
    need_gpu()
    import paper_2307_09582_amd as glu

    return glu


def random_theta(H, W, s, k, seed):
    """Random valid Theta: both endpoints inside the truncated window."""
    rng = np.random.default_rng(seed)
    h, w = -(-H // s), -(-W // s)
    r = k // 2
    ys, xs = np.mgrid[0:H, 0:W]
    qy, qx = ys // s, xs // s

    def pick():
        cy = np.clip(qy + rng.integers(-r, r + 1, (H, W)), 0, h - 1)
        cx = np.clip(qx + rng.integers(-r, r + 1, (H, W)), 0, w - 1)
        return (cy - qy + r) * k + (cx - qx + r), cy * w + cx

    oa, a = pick()
    ob, b = pick()
    code = (oa * k * k + ob).astype(np.uint16)
    alpha = rng.uniform(0, 1, (H, W)).astype(np.float32)
    alpha[rng.uniform(size=(H, W)) < 0.1] = 1.0
    same = rng.uniform(size=(H, W)) < 0.1
    code[same] = (oa[same] * k * k + oa[same]).astype(np.uint16)
    b = np.where(same, a, b)
    return code, alpha, a, b


def _check(glu, H, W, s, k, C, seed, t_dtype=torch.float32):
    log_case(test="backward", H=H, W=W, s=s, k=k, C=C, seed=seed)
    code, alpha, a, b = random_theta(H, W, s, k, seed)
    rng = np.random.default_rng(seed + 1)
    h, w = -(-H // s), -(-W // s)
    T = rng.uniform(0, 1, (h, w, C)).astype(np.float32)
    if t_dtype == torch.float16:
        T = T.astype(np.float16)
    G = rng.normal(0, 1, (H, W, C)).astype(np.float32)
    th = glu.Theta(dev(code.view(np.int16)), dev(alpha))
    gT, ga = glu.apply_backward(th, dev(T), dev(G), s, k)
    gT, ga = host(gT), host(ga)
    da_ref, dT_ref = O.apply_backward(a.ravel(), b.ravel(), alpha.ravel(), T.astype(np.float64), G.astype(np.float64))
    da_ref = da_ref.reshape(H, W)
    assert np.all(np.abs(ga - da_ref) <= 1e-5 * (1 + np.abs(da_ref))), float(np.abs(ga - da_ref).max())
    # per-cell L1 mass of the summed contributions bounds the rounding of the sum
    mass = np.zeros((h * w, C))
    Gf = np.abs(G.reshape(-1, C).astype(np.float64))
    np.add.at(mass, a.ravel(), alpha.ravel()[:, None] * Gf)
    np.add.at(mass, b.ravel(), (1 - alpha.ravel())[:, None] * Gf)
    err = np.abs(gT.reshape(-1, C) - dT_ref.reshape(-1, C))
    assert np.all(err <= 1e-5 * mass + 1e-12), float((err / (mass + 1e-30)).max())
    # bitwise determinism
    gT2, ga2 = glu.apply_backward(th, dev(T), dev(G), s, k)
    assert np.array_equal(host(gT2), gT) and np.array_equal(host(ga2), ga)
    # only one of the two outputs
    gT3, ga3 = glu.apply_backward(th, dev(T), dev(G), s, k, need_alpha=False)
    assert ga3 is None and np.array_equal(host(gT3), gT)
    gT4, ga4 = glu.apply_backward(th, dev(T), dev(G), s, k, need_T_low=False)
    assert gT4 is None and np.array_equal(host(ga4), ga)


@pytest.mark.parametrize(
    "H,W,s,k,C",
    [
        (256, 320, 8, 3, 3),
        (100, 77, 3, 3, 4),
        (64, 72, 4, 5, 1),
        (130, 170, 16, 3, 2),
        (33, 29, 2, 7, 3),
        (7, 5, 8, 3, 1),
        (512, 512, 8, 3, 3),
        (96, 96, 32, 3, 3),
        (72, 100, 4, 3, 4),
        (70, 91, 8, 3, 3),
        (40, 36, 12, 3, 3),
        (200, 260, 64, 3, 3),
        (300, 260, 128, 3, 1),
        (33, 2100, 8, 3, 2),
        (100, 130, 20, 3, 2),
        (520, 300, 256, 3, 3),
        (24, 20, 512, 3, 3),
        (64, 90, 2, 3, 3),
        (31, 47, 3, 3, 3),
        (70, 100, 6, 3, 1),
        (55, 73, 10, 3, 3),
        (60, 80, 9, 3, 2),
        (29, 41, 2, 3, 4),
        (72, 100, 4, 5, 3),
        (64, 80, 8, 5, 4),
        (96, 96, 16, 5, 2),
        (50, 70, 12, 5, 1),
        (41, 67, 8, 5, 3),
    ],
)
def test_backward_parity(H, W, s, k, C):
    _check(_glu(), H, W, s, k, C, seed=H + 7 * W + s)


def test_backward_half_T_low():
    _check(_glu(), 120, 136, 8, 3, 3, seed=5, t_dtype=torch.float16)


def test_backward_fd_on_crops():
    """FP64 central finite differences of the oracle loss on 64 x 64 crops,
    against the GPU gradients of the same quadratic loss."""
    glu = _glu()
    H = W = 1024
    s, k = 8, 3
    I = synth.voronoi(H, W, n_cells=150, n_dots=40, dot_px=(1, 3), seed=5)
    L = O.downsample_point(I, s)
    T = synth.lr_op_f1(L).astype(np.float32)
    th = glu.search(dev(I), dev(L), s, k)
    code, alpha = host(th.code), host(th.alpha)
    from tests.parity import decode_codes

    a, b, ok = decode_codes(code, H, W, s, k, np.arange(H * W))
    assert ok.all()
    rng = np.random.default_rng(5)
    target = (synth.lr_op_f1(I) + rng.normal(0, 0.01, (H, W, 3))).astype(np.float32)
    for ci in range(4):
        y0 = int(rng.integers(0, (H - 64) // s)) * s
        x0 = int(rng.integers(0, (W - 64) // s)) * s
        mask = np.zeros((H, W, 1), np.float32)
        mask[y0 : y0 + 64, x0 : x0 + 64] = 1.0
        out = host(glu.apply(th, dev(T), s, k))
        G = (2.0 * (out - target) * mask).astype(np.float32)
        gT, ga = glu.apply_backward(th, dev(T), dev(G), s, k)
        gT, ga = host(gT), host(ga)
        pix = np.flatnonzero(mask[..., 0].ravel())
        tgt = target.reshape(-1, 3)[pix].astype(np.float64)

        def loss(Tl, al):
            o = O.apply(a.ravel()[pix], b.ravel()[pix], al[pix], Tl)
            return float(((o - tgt) ** 2).sum())

        al64 = alpha.ravel().astype(np.float64)
        T64 = T.astype(np.float64)
        eps = 1e-6
        # LR entries the crop touches
        cells = np.unique(np.concatenate([a.ravel()[pix], b.ravel()[pix]]))
        for q in rng.choice(cells, 6, replace=False):
            for c in range(3):
                Tp, Tm = T64.copy(), T64.copy()
                Tp.reshape(-1, 3)[q, c] += eps
                Tm.reshape(-1, 3)[q, c] -= eps
                fd = (loss(Tp, al64) - loss(Tm, al64)) / (2 * eps)
                g = gT.reshape(-1, 3)[q, c]
                assert abs(g - fd) <= 1e-5 * (1 + abs(fd)) + 1e-4, (q, c, g, fd)
        for p in rng.choice(pix, 8, replace=False):
            ap, am = al64.copy(), al64.copy()
            ap[p] += eps
            am[p] -= eps
            fd = (loss(T64, ap) - loss(T64, am)) / (2 * eps)
            assert abs(ga.ravel()[p] - fd) <= 1e-5 * (1 + abs(fd)) + 1e-5, (p, ga.ravel()[p], fd)


def test_autograd_function_matches_torch_reference():
    """GluApply inside a loss: gradients equal a float64 CPU autograd reference
    built from index_select."""
    glu = _glu()
    H, W, s, k = 96, 128, 8, 3
    code, alpha, a, b = random_theta(H, W, s, k, 17)
    rng = np.random.default_rng(17)
    T = rng.uniform(0, 1, (H // s, W // s, 3)).astype(np.float32)
    target = rng.uniform(0, 1, (H, W, 3)).astype(np.float32)
    al_t = dev(alpha).requires_grad_(True)
    T_t = dev(T).requires_grad_(True)
    out = glu.glu_apply_autograd(al_t, T_t, dev(code.view(np.int16)), s, k)
    loss = ((out - dev(target)) ** 2).mean()
    loss.backward()
    # reference in float64 on the CPU
    Tr = torch.tensor(T.reshape(-1, 3), dtype=torch.float64, requires_grad=True)
    ar = torch.tensor(alpha.ravel(), dtype=torch.float64, requires_grad=True)
    o = ar[:, None] * Tr.index_select(0, torch.tensor(a.ravel())) + (1 - ar[:, None]) * Tr.index_select(
        0, torch.tensor(b.ravel()))
    lr = ((o - torch.tensor(target.reshape(-1, 3), dtype=torch.float64)) ** 2).mean()
    lr.backward()
    np.testing.assert_allclose(host(al_t.grad).ravel(), ar.grad.numpy(), rtol=1e-4, atol=1e-9)
    np.testing.assert_allclose(host(T_t.grad).reshape(-1, 3), Tr.grad.numpy(), rtol=1e-4, atol=1e-9)


@pytest.mark.parametrize("H,W,s,k,C,step", [(96, 136, 8, 3, 3, 1), (50, 70, 4, 5, 2, 2), (33, 29, 3, 3, 1, 1),
                                              (40, 62, 2, 3, 3, 1)])
def test_batched_apply_and_backward_equal_per_image(H, W, s, k, C, step):
    """glu_apply_batched / glu_apply_backward_batched give bitwise the results
    of per-image calls, also for a strided view of a larger batch."""
    glu = _glu()
    log_case(test="batched_apply_backward", H=H, W=W, s=s, k=k, C=C, step=step)
    B = 3
    h, w = -(-H // s), -(-W // s)
    rng = np.random.default_rng(H + W + s)
    codes, alphas = [], []
    for b in range(B * step):
        code, alpha, _, _ = random_theta(H, W, s, k, seed=100 + b)
        codes.append(code.view(np.int16))
        alphas.append(alpha)
    code = dev(np.stack(codes))[::step]
    alpha = dev(np.stack(alphas))[::step]
    T = dev(rng.uniform(0, 1, (B * step, h, w, C)).astype(np.float32))[::step]
    G = dev(rng.normal(0, 1, (B * step, H, W, C)).astype(np.float32))[::step]
    th = glu.Theta(code, alpha)
    out = glu.apply(th, T, s, k)
    gT, ga = glu.apply_backward(th, T, G, s, k)
    for b in range(B):
        thb = glu.Theta(code[b].contiguous(), alpha[b].contiguous())
        ob = glu.apply(thb, T[b].contiguous(), s, k)
        gTb, gab = glu.apply_backward(thb, T[b].contiguous(), G[b].contiguous(), s, k)
        assert torch.equal(out[b], ob)
        assert torch.equal(gT[b], gTb) and torch.equal(ga[b], gab)


def test_batched_autograd_matches_loop():
    """GluApply over a (B, H, W) batch: one forward and one backward launch per
    pass, gradients equal to the per-image autograd calls."""
    glu = _glu()
    log_case(test="batched_autograd")
    B, H, W, s, k, C = 4, 64, 80, 8, 3, 3
    h, w = H // s, W // s
    codes = [random_theta(H, W, s, k, seed=200 + b)[0].view(np.int16) for b in range(B)]
    code = dev(np.stack(codes))
    rng = np.random.default_rng(7)
    alpha = dev(rng.uniform(0, 1, (B, H, W)).astype(np.float32)).requires_grad_(True)
    T = dev(rng.uniform(0, 1, (B, h, w, C)).astype(np.float32)).requires_grad_(True)
    target = dev(rng.uniform(0, 1, (B, H, W, C)).astype(np.float32))
    loss = ((glu.glu_apply_autograd(alpha, T, code, s, k) - target) ** 2).mean()
    loss.backward()
    ga, gT = alpha.grad.clone(), T.grad.clone()
    for b in range(B):
        a1 = alpha.detach()[b].clone().requires_grad_(True)
        T1 = T.detach()[b].clone().requires_grad_(True)
        l1 = ((glu.glu_apply_autograd(a1, T1, code[b], s, k) - target[b]) ** 2).sum() / target.numel()
        l1.backward()
        assert torch.allclose(a1.grad, ga[b], rtol=1e-6, atol=1e-12)
        assert torch.allclose(T1.grad, gT[b], rtol=1e-6, atol=1e-12)


@pytest.mark.parametrize("H,W,s,k,C", [(64, 72, 8, 3, 3), (37, 41, 4, 5, 2), (20, 9, 4, 3, 1), (8, 8, 8, 3, 3),
                                       (45, 52, 4, 7, 4), (40, 36, 3, 9, 3), (70, 6, 2, 5, 1), (5, 40, 8, 3, 3)])
def test_border_and_invalid_codes_follow_the_clamp_rule(H, W, s, k, C):
    """Codes the search never writes: window positions outside the LR image
    (at its borders) and codes above k^4 - 1.  The apply reads the nearest
    in-image cell (clamped row and column; a code above k^4 - 1 counts as
    k^4 - 1), and the backward sends each gradient to the same cell, so both
    match the oracle's Eq. 1 and its gradient with those cells."""
    glu = _glu()
    log_case(test="backward_clamp_rule", H=H, W=W, s=s, k=k, C=C)
    rng = np.random.default_rng(H * 31 + W)
    h, w = -(-H // s), -(-W // s)
    r, K2 = k // 2, k * k
    oa = rng.integers(0, K2, (H, W))
    ob = rng.integers(0, K2, (H, W))
    code = (oa * K2 + ob).astype(np.uint16)
    code[rng.random((H, W)) < 0.1] = 0xFFFF
    alpha = rng.random((H, W)).astype(np.float32)
    T = rng.random((h, w, C)).astype(np.float32)
    G = rng.normal(0, 1, (H, W, C)).astype(np.float32)
    # the rule, written out: clamp the code, then each cell into the image
    cd = np.minimum(code.astype(np.int64), K2 * K2 - 1)
    ys, xs = np.mgrid[0:H, 0:W]
    qy, qx = ys // s, xs // s

    def cell(o):
        cy = np.clip(qy + o // k - r, 0, h - 1)
        cx = np.clip(qx + o % k - r, 0, w - 1)
        return (cy * w + cx).ravel()

    a, b = cell(cd // K2), cell(cd % K2)
    th = glu.Theta(dev(code.view(np.int16)), dev(alpha))
    out = host(glu.apply(th, dev(T), s, k))
    ref = O.apply(a, b, alpha.ravel(), T).reshape(H, W, C)
    assert np.abs(out - ref).max() <= 1e-5
    gT, ga = glu.apply_backward(th, dev(T), dev(G), s, k)
    gT, ga = host(gT), host(ga)
    da_ref, dT_ref = O.apply_backward(a, b, alpha.ravel(), T, G.reshape(-1, C))
    assert np.all(np.abs(ga.ravel() - da_ref) <= 1e-5 * (1 + np.abs(da_ref)))
    mass = np.zeros((h * w, C))
    Gf = np.abs(G.reshape(-1, C).astype(np.float64))
    np.add.at(mass, a, alpha.ravel()[:, None] * Gf)
    np.add.at(mass, b, (1 - alpha.ravel())[:, None] * Gf)
    err = np.abs(gT.reshape(-1, C) - dT_ref.reshape(-1, C))
    assert np.all(err <= 1e-5 * mass + 1e-12), float((err / (mass + 1e-30)).max())
