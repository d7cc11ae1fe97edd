"""GPU parity of glu_search / glu_apply / glu_search_apply against the oracle."""
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


def _inputs(H, W, s, seed, n_cells, n_dots, dot_px=(1, 3), down="point", C=3, lr_op="f1"):
    I = synth.voronoi(H, W, n_cells=n_cells, n_dots=n_dots, dot_px=dot_px, sigma=0.01, seed=seed)
    if down == "point":
        L = O.downsample_point(I, s)
    else:
        L = O.downsample_box(I, s).astype(np.float32)
    if lr_op == "f1":
        T = synth.lr_op_f1(L)
    else:
        T = synth.lr_op_f2(L)
    if C == 1:
        T = T[..., :1]
    elif C == 2:
        T = T[..., :2]
    elif C == 4:
        T = np.concatenate([T, T[..., :1] * 0.5], axis=-1)
    return I, np.ascontiguousarray(L.astype(np.float32)), np.ascontiguousarray(T.astype(np.float32))


def _run_and_check(glu, I, L, T, s, k, mode, eps=1e-3, dtype=torch.float32, fused_too=True):
    npd = np.float16 if dtype == torch.float16 else np.float32
    I = I.astype(npd)
    L = L.astype(npd)
    T = T.astype(npd)
    dI, dL, dT = dev(I), dev(L), dev(T)
    th, err = glu.search(dI, dL, s, k, eps, mode, return_err=True)
    out = glu.apply(th, dT, s, k)
    code, alpha, e, That = host(th.code), host(th.alpha), host(err), host(out)
    rep = check_search(I, L, s, k, eps, mode, code, alpha, err=e, T_low=T, T_hat=That, out_dtype=npd)
    if fused_too:
        out2, th2, err2 = glu.search_apply(dI, dL, dT, s, k, eps, mode, return_err=True)
        # the fused pass gives bitwise the same Theta, E and T_hat as the two calls
        assert np.array_equal(host(th2.code), code)
        assert np.array_equal(host(th2.alpha).view(np.uint32), alpha.view(np.uint32))
        assert np.array_equal(host(err2).view(np.uint32), e.view(np.uint32))
        assert np.array_equal(host(out2), That)
        out3, th3 = glu.search_apply(dI, dL, dT, s, k, eps, mode, store_theta=False)
        assert th3 is None
        assert np.array_equal(host(out3), That)
    return rep


@pytest.mark.parametrize("mode", ["exhaustive", "fast"])
def test_plain_512_box4(mode):
    """Plain GLU on a 512 x 512 Voronoi image, box x4 to 128 x 128, 3 x 3 window."""
    glu = _glu()
    log_case(test="plain_512_box4", mode=mode)
    I, L, T = _inputs(512, 512, 4, seed=1, n_cells=64, n_dots=20, dot_px=(2, 4), down="box")
    rep = _run_and_check(glu, I, L, T, 4, 3, mode)
    print(rep)


CASES = [
    # H, W, s, k, C, mode, dtype
    (37, 53, 4, 3, 3, "exhaustive", "f32"),
    (64, 96, 8, 3, 1, "fast", "f32"),
    (29, 31, 3, 3, 4, "exhaustive", "f32"),
    (29, 31, 3, 3, 2, "fast", "f32"),
    (50, 70, 2, 5, 3, "exhaustive", "f32"),
    (72, 88, 4, 5, 3, "exhaustive", "f32"),
    (72, 88, 8, 5, 3, "fast", "f32"),
    (40, 40, 8, 1, 3, "exhaustive", "f32"),
    (40, 40, 8, 1, 3, "fast", "f32"),
    (41, 39, 4, 7, 3, "exhaustive", "f32"),
    (41, 39, 4, 7, 3, "fast", "f32"),
    (23, 17, 16, 3, 3, "exhaustive", "f32"),
    (5, 7, 8, 3, 3, "exhaustive", "f32"),
    (1, 1, 1, 3, 1, "exhaustive", "f32"),
    (16, 24, 1, 3, 3, "exhaustive", "f32"),
    (16, 24, 1, 3, 3, "fast", "f32"),
    (130, 170, 16, 3, 3, "exhaustive", "f32"),
    (200, 264, 8, 3, 3, "exhaustive", "f16"),
    (200, 264, 8, 3, 3, "fast", "f16"),
    (57, 61, 4, 3, 1, "exhaustive", "f16"),
    (96, 100, 12, 3, 3, "exhaustive", "f32"),
    (48, 48, 4, 9, 3, "exhaustive", "f32"),
    (30, 45, 3, 3, 3, "exhaustive", "f16"),
    (30, 45, 2, 3, 1, "fast", "f16"),
    (40, 72, 4, 3, 4, "fast", "f16"),
    (40, 72, 4, 3, 2, "exhaustive", "f16"),
    (128, 192, 32, 3, 3, "exhaustive", "f32"),
    (300, 400, 64, 3, 3, "exhaustive", "f32"),
    (260, 520, 128, 3, 3, "fast", "f32"),
    (200, 200, 64, 5, 1, "fast", "f32"),
    (61, 75, 6, 3, 3, "exhaustive", "f32"),
    (61, 75, 6, 3, 3, "fast", "f32"),
    (44, 58, 10, 3, 2, "exhaustive", "f16"),
    (70, 90, 6, 5, 3, "exhaustive", "f32"),
    (37, 41, 2, 3, 4, "exhaustive", "f32"),
    (80, 100, 9, 3, 3, "exhaustive", "f32"),
    (80, 100, 9, 3, 3, "fast", "f16"),
    (33, 47, 3, 5, 3, "exhaustive", "f32"),
    (72, 88, 8, 5, 3, "exhaustive", "f32"),
    (96, 112, 16, 5, 2, "exhaustive", "f16"),
    (41, 67, 8, 5, 1, "exhaustive", "f32"),
    # float32 fast tiles with strips of 2 or 3 pixels (per-pixel staged T_hat)
    (37, 41, 2, 3, 4, "fast", "f32"),
    (50, 66, 2, 3, 1, "fast", "f32"),
    (64, 200, 2, 3, 3, "fast", "f32"),
    (45, 63, 3, 3, 4, "fast", "f32"),
    (33, 36, 6, 3, 1, "fast", "f32"),
    (97, 200, 6, 3, 3, "fast", "f32"),
]


@pytest.mark.parametrize("H,W,s,k,C,mode,dt", CASES)
def test_shapes(H, W, s, k, C, mode, dt):
    glu = _glu()
    log_case(test="shapes", H=H, W=W, s=s, k=k, C=C, mode=mode, dt=dt)
    I, L, T = _inputs(H, W, s, seed=H * 131 + W, n_cells=max(4, H * W // 400), n_dots=3, C=C)
    dtype = torch.float16 if dt == "f16" else torch.float32
    _run_and_check(glu, I, L, T, s, k, mode, dtype=dtype)


@pytest.mark.parametrize("mode", ["exhaustive", "fast"])
def test_eps_zero_well_separated(mode):
    """eps = 0 (no regulariser) on a well-separated palette image."""
    glu = _glu()
    rng = np.random.default_rng(3)
    pal = rng.uniform(0, 1, (6, 3))
    lab = rng.integers(0, 6, (20, 28))
    I = np.repeat(np.repeat(pal[lab], 4, 0), 4, 1)[:75, :106].astype(np.float32)
    I = np.clip(I + rng.normal(0, 0.02, I.shape), 0, 1).astype(np.float32)
    L = O.downsample_point(I, 4)
    T = synth.lr_op_f1(L).astype(np.float32)
    _run_and_check(glu, I, L, T, 4, 3, mode, eps=0.0)


@pytest.mark.parametrize("mode", ["exhaustive", "fast"])
def test_nearest_copy_exact_zero(mode):
    """HR = s x s replicas of LR: E is exactly 0 and T_hat nearest-neighbour."""
    glu = _glu()
    rng = np.random.default_rng(7)
    s = 8
    L = rng.uniform(0, 1, (30, 41, 3)).astype(np.float32)
    I = np.ascontiguousarray(np.repeat(np.repeat(L, s, 0), s, 1)[:235, :321])
    T = rng.uniform(0, 1, (30, 41, 2)).astype(np.float32)
    out, th, err = glu.search_apply(dev(I), dev(L), dev(T), s, 3, 1e-3, mode, return_err=True)
    assert np.all(host(err) == 0.0)
    nn = np.repeat(np.repeat(T, s, 0), s, 1)[:235, :321]
    assert np.array_equal(host(out), nn)


def test_constant_image():
    glu = _glu()
    I = np.broadcast_to(np.array([0.3, 0.6, 0.2], np.float32), (70, 90, 3)).copy()
    L = O.downsample_point(I, 8)
    T = np.full(L.shape[:2] + (1,), 0.7, np.float32)
    for mode in ("exhaustive", "fast"):
        out, th, err = glu.search_apply(dev(I), dev(L), dev(T), 8, 3, 1e-3, mode, return_err=True)
        assert np.all(host(err) == 0.0)
        assert np.all(host(out) == np.float32(0.7))


def test_empty_image_is_a_no_op():
    glu = _glu()
    I = torch.empty((0, 16, 3), device="cuda")
    L = torch.empty((0, 2, 3), device="cuda")
    th = glu.search(I, L, 8, 3)
    assert th.code.shape == (0, 16)


def test_determinism_and_theta_expand():
    glu = _glu()
    I, L, T = _inputs(160, 200, 8, seed=9, n_cells=30, n_dots=8)
    dI, dL = dev(I), dev(L)
    th1, e1 = glu.search(dI, dL, 8, 3, return_err=True)
    th2, e2 = glu.search(dI, dL, 8, 3, return_err=True)
    assert torch.equal(th1.code, th2.code) and torch.equal(th1.alpha, th2.alpha) and torch.equal(e1, e2)
    a, b = glu.theta_expand(th1, 8, 3)
    from tests.parity import decode_codes

    pix = np.arange(160 * 200)
    ra, rb, ok = decode_codes(host(th1.code), 160, 200, 8, 3, pix)
    assert ok.all()
    assert np.array_equal(host(a).ravel(), ra) and np.array_equal(host(b).ravel(), rb)


@pytest.mark.parametrize("mode", ["point", "box"])
def test_downsample(mode):
    glu = _glu()
    I = synth.voronoi(67, 93, n_cells=10, n_dots=4, seed=5)
    out = host(glu.downsample(dev(I), 8, mode))
    if mode == "point":
        assert np.array_equal(out, O.downsample_point(I, 8))
    else:
        np.testing.assert_allclose(out, O.downsample_box(I, 8), atol=1e-6)


def test_padded_rows_and_views():
    """Row strides larger than W*C (views into wider buffers) give the same result."""
    glu = _glu()
    I, L, T = _inputs(64, 80, 4, seed=21, n_cells=12, n_dots=4)
    big = np.zeros((64, 84, 3), np.float32)
    big[:, :80] = I
    dI = dev(big)[:, :80]
    th, e = glu.search(dI, dev(L), 4, 3, return_err=True)
    th0, e0 = glu.search(dev(I), dev(L), 4, 3, return_err=True)
    assert torch.equal(th.code, th0.code) and torch.equal(th.alpha, th0.alpha)


@pytest.mark.parametrize("mode", ["exhaustive", "fast"])
def test_padded_theta_err_and_grad_alpha(mode):
    """E and grad_alpha share Theta's row stride in the C ABI: with a padded
    Theta the binding lays them out (or checks them) with that stride, the
    values equal those of a dense Theta and the padding is never written."""
    glu = _glu()
    log_case(test="padded_theta", mode=mode)
    H, W, s, pad = 64, 100, 4, 12
    I, L, T = _inputs(H, W, s, seed=23, n_cells=10, n_dots=4)
    dI, dL, dT = dev(I), dev(L), dev(T)

    def padded_theta():
        code = torch.full((H, W + pad), -7, dtype=torch.int16, device="cuda")
        alpha = torch.full((H, W + pad), 7.0, dtype=torch.float32, device="cuda")
        return glu.Theta(code[:, :W], alpha[:, :W]), code, alpha

    th0, e0 = glu.search(dI, dL, s, 3, 1e-3, mode, return_err=True)
    thp, code_p, alpha_p = padded_theta()
    _, ep = glu.search(dI, dL, s, 3, 1e-3, mode, return_err=True, theta=thp)
    assert ep.stride(0) == W + pad
    assert torch.equal(thp.code, th0.code) and torch.equal(thp.alpha, th0.alpha) and torch.equal(ep, e0)
    assert bool((code_p[:, W:] == -7).all()) and bool((alpha_p[:, W:] == 7.0).all())
    # a caller's buffer must have Theta's row stride
    with pytest.raises(ValueError):
        glu.search(dI, dL, s, 3, 1e-3, mode, return_err=True, theta=thp, err=torch.empty((H, W), device="cuda"))
    eb = torch.full((H, W + pad), 9.0, device="cuda")
    glu.search(dI, dL, s, 3, 1e-3, mode, return_err=True, theta=thp, err=eb[:, :W])
    assert torch.equal(eb[:, :W], e0) and bool((eb[:, W:] == 9.0).all())

    out0, _, ef0 = glu.search_apply(dI, dL, dT, s, 3, 1e-3, mode, return_err=True)
    thq, _, _ = padded_theta()
    outq, _, efq = glu.search_apply(dI, dL, dT, s, 3, 1e-3, mode, return_err=True, theta=thq)
    assert efq.stride(0) == W + pad and torch.equal(efq, ef0) and torch.equal(outq, out0)

    G = torch.randn((H, W, 3), device="cuda", generator=torch.Generator("cuda").manual_seed(24))
    gT0, ga0 = glu.apply_backward(th0, dT, G, s, 3)
    gTp, gap = glu.apply_backward(thp, dT, G, s, 3)
    assert gap.stride(0) == W + pad and torch.equal(gap, ga0) and torch.equal(gTp, gT0)
    gb = torch.full((H, W + pad), 5.0, device="cuda")
    glu.apply_backward(thp, dT, G, s, 3, out_alpha=gb[:, :W])
    assert torch.equal(gb[:, :W], ga0) and bool((gb[:, W:] == 5.0).all())
    with pytest.raises(ValueError):
        glu.apply_backward(thp, dT, G, s, 3, out_alpha=torch.empty((H, W), device="cuda"))


@pytest.mark.parametrize("mode", ["exhaustive", "fast"])
def test_full_4k_x8_sampled(mode):
    """The 3840 x 2160 x8 workload, in the launch configuration the benchmark
    times (fused search + apply), checked on sampled pixels: 20000 random
    pixels plus every pixel of the first and last tile rows and columns."""
    glu = _glu()
    log_case(test="full_4k_x8_sampled", mode=mode)
    H, W, s = 2160, 3840, 8
    I = synth.voronoi(H, W, n_cells=1000, n_dots=400, dot_px=(1, 3), seed=3)
    L = O.downsample_point(I, s)
    T = synth.lr_op_f1(L).astype(np.float32)
    out, th, err = glu.search_apply(dev(I), dev(L), dev(T), s, 3, 1e-3, mode, return_err=True)
    rng = np.random.default_rng(0)
    pix = [rng.choice(H * W, 20000, replace=False)]
    ys, xs = np.mgrid[0:H, 0:W]
    edge = (ys < 16) | (ys >= H - 16) | (xs < 64) | (xs >= W - 64)
    pix.append(np.flatnonzero(edge.ravel())[::7])
    pix = np.unique(np.concatenate(pix))
    rep = check_search(I, L, s, 3, 1e-3, mode, host(th.code), host(th.alpha), err=host(err), pixels=pix,
                       T_low=T, T_hat=host(out))
    print(rep)


@pytest.mark.parametrize("mode", ["exhaustive", "fast"])
def test_full_4k_x8_every_pixel_bench_launch(mode, oracle_pool):
    """The benchmark's own frame and launch, every pixel: frame 0 of the
    3840 x 2160 scene (1000 cells, 400 dots of 1-3 px, canvas 177 px wider,
    sigma 0.01, float32), regular-grid x8, target f1, one fused
    search + apply writing Theta and T_hat (no E), checked on all 8294400
    pixels against the oracle (its search run by a pool of host processes)."""
    glu = _glu()
    log_case(test="full_4k_x8_every_pixel", mode=mode)
    H, W, s = 2160, 3840, 8
    I = synth.make_scene(H, W, 1000, 400, (1, 3), seed=3, canvas_extra=177).frame(0, sigma=0.01, dtype=np.float32)
    L = O.downsample_point(I, s)
    T = synth.lr_op_f1(L).astype(np.float32)
    dI = dev(I)
    assert np.array_equal(host(glu.downsample(dI, s, "point")), L)
    th = glu.empty_theta(H, W)
    out = torch.empty((H, W, 3), dtype=torch.float32, device="cuda")
    glu.search_apply(dI, dev(L), dev(T), s, 3, 1e-3, mode, theta=th, out=out)
    code, alpha, That = host(th.code), host(th.alpha), host(out)
    ref = oracle_pool.search(I, L, s, 3, 1e-3, mode)
    rep = check_search(I, L, s, 3, 1e-3, mode, code, alpha, T_low=T, T_hat=That, ref=ref)
    print(mode, dict(rep), flush=True)


@pytest.mark.parametrize("s,mode", [(2, "exhaustive"), (3, "exhaustive"), (4, "exhaustive"), (2, "fast"),
                                    (3, "fast"), (4, "fast")])
def test_large_image_small_ratio_every_pixel(s, mode, oracle_pool):
    """A 1152 x 1280 scene with the cell and dot density of the 4K scene, at
    s = 2, 3, 4: large enough that a single-image launch keeps its default
    strips (2, 3 and 4 pixels), so the exhaustive search runs without the
    pair table, its window in registers.
    Every pixel of Theta, E (a separate search) and the fused T_hat against
    the oracle, which runs in a pool of host processes."""
    glu = _glu()
    log_case(test="large_image_small_ratio", s=s, mode=mode)
    H, W = 1152, 1280
    I = synth.make_scene(H, W, 180, 70, (1, 3), seed=5).frame(0, sigma=0.01, dtype=np.float32)
    L = O.downsample_point(I, s)
    T = synth.lr_op_f1(L).astype(np.float32)
    dI, dL = dev(I), dev(L)
    th = glu.empty_theta(H, W)
    out = torch.empty((H, W, 3), dtype=torch.float32, device="cuda")
    glu.search_apply(dI, dL, dev(T), s, 3, 1e-3, mode, theta=th, out=out)
    th2, err = glu.search(dI, dL, s, 3, 1e-3, mode, return_err=True)
    code, alpha = host(th.code), host(th.alpha)
    assert np.array_equal(code, host(th2.code)) and np.array_equal(alpha, host(th2.alpha))
    ref = oracle_pool.search(I, L, s, 3, 1e-3, mode)
    rep = check_search(I, L, s, 3, 1e-3, mode, code, alpha, err=host(err), T_low=T, T_hat=host(out), ref=ref)
    print(s, mode, dict(rep), flush=True)


def _random_theta(H, W, s, k, rng):
    """Codes of random pairs inside each pixel's border-truncated window and
    random weights in [0, 1]; returns (code, alpha, a, b) with absolute LR
    indices a, b."""
    h, w = -(-H // s), -(-W // s)
    r = k // 2
    ys, xs = np.mgrid[0:H, 0:W]
    qy, qx = ys // s, xs // s

    def offset():
        lo_y, hi_y = np.maximum(-r, -qy), np.minimum(r, h - 1 - qy)
        lo_x, hi_x = np.maximum(-r, -qx), np.minimum(r, w - 1 - qx)
        dy = lo_y + np.floor(rng.random((H, W)) * (hi_y - lo_y + 1)).astype(np.int64)
        dx = lo_x + np.floor(rng.random((H, W)) * (hi_x - lo_x + 1)).astype(np.int64)
        return (dy + r) * k + (dx + r), (qy + dy) * w + (qx + dx)

    oa, a = offset()
    ob, b = offset()
    code = (oa * k * k + ob).astype(np.uint16).view(np.int16)
    alpha = rng.random((H, W)).astype(np.float32)
    alpha[0, 0] = 0.0
    alpha[-1, -1] = 1.0
    return code, alpha, a, b


APPLY_CASES = [
    # H, W, s, k, C, dtype, extra row padding (pixels), column offset of the output view
    (96, 1000, 8, 3, 3, "f32", 0, 0),
    (64, 520, 8, 3, 3, "f32", 4, 1),
    (16, 4160, 8, 3, 3, "f32", 4, 0),
    (70, 300, 4, 5, 4, "f32", 0, 0),
    (50, 200, 16, 3, 3, "f32", 0, 0),
    (20, 700, 1, 3, 3, "f32", 0, 0),
    (25, 77, 5, 7, 3, "f32", 0, 0),
    (33, 250, 3, 3, 3, "f16", 0, 0),
    (33, 250, 2, 3, 1, "f16", 0, 0),
    (40, 130, 4, 3, 2, "f16", 0, 0),
    (40, 136, 8, 3, 3, "f16", 2, 1),
    (9, 2100, 12, 3, 1, "f32", 0, 0),
]


@pytest.mark.parametrize("H,W,s,k,C,dt,pad,off", APPLY_CASES)
def test_apply_random_theta(H, W, s, k, C, dt, pad, off):
    """glu_apply with random valid Theta against Eq. 1 in float64, into
    dense outputs and into views whose rows are padded or misaligned."""
    glu = _glu()
    log_case(test="apply_random_theta", H=H, W=W, s=s, k=k, C=C, dt=dt, pad=pad, off=off)
    rng = np.random.default_rng(H * 7919 + W * 31 + s)
    code, alpha, a, b = _random_theta(H, W, s, k, rng)
    h, w = -(-H // s), -(-W // s)
    npd = np.float16 if dt == "f16" else np.float32
    T = rng.random((h, w, C)).astype(npd)
    th = glu.Theta(dev(code), dev(alpha))
    big = torch.full((H, W + pad + off, C), float("nan"), dtype=torch.float16 if dt == "f16" else torch.float32,
                     device="cuda")
    view = big[:, off:off + W]
    out = glu.apply(th, dev(T), s, k, out=view)
    got = host(out).astype(np.float64)
    ref = O.apply(a, b, alpha, T)
    if dt == "f16":
        tol = np.spacing(np.abs(ref).astype(np.float16)).astype(np.float64) + 1e-5
    else:
        tol = 1e-5
    bad = np.abs(got - ref) > tol
    assert not bad.any(), "apply mismatch at %d values, first %s" % (int(bad.sum()), np.argwhere(bad)[0])
    rest = host(big)
    if off:
        assert np.isnan(rest[:, :off]).all()
    if pad:
        assert np.isnan(rest[:, off + W:]).all()


@pytest.mark.parametrize("H,W,s,k,C", [(64, 80, 4, 3, 3), (37, 53, 5, 5, 1), (9, 7, 16, 3, 3), (40, 40, 4, 1, 3),
                                        (130, 170, 8, 3, 2)])
def test_no_degenerate_flag(H, W, s, k, C):
    """GLU_FLAG_NO_DEGENERATE: the pairs i < j alone, against the oracle's
    literal candidate set, through search, the fused pass and a batch plan;
    on noise-free inputs, where the flag changes the result."""
    glu = _glu()
    log_case(test="no_degenerate", H=H, W=W, s=s, k=k, C=C)
    I = synth.voronoi(H, W, n_cells=max(4, H * W // 300), n_dots=2, dot_px=(1, 3), sigma=0.0, seed=H * 3 + W)
    L = np.ascontiguousarray(O.downsample_point(I, s).astype(np.float32))
    T = np.ascontiguousarray(synth.lr_op_f1(L)[..., :C].astype(np.float32))
    dI, dL, dT = dev(I.astype(np.float32)), dev(L), dev(T)
    th, err = glu.search(dI, dL, s, k, 1e-3, "exhaustive", return_err=True, degenerate=False)
    out = glu.apply(th, dT, s, k)
    code, alpha, e = host(th.code), host(th.alpha), host(err)
    check_search(I.astype(np.float32), L, s, k, 1e-3, "exhaustive", code, alpha, err=e, T_low=T, T_hat=host(out),
                 degenerate=False)
    out2, th2, err2 = glu.search_apply(dI, dL, dT, s, k, 1e-3, "exhaustive", return_err=True, degenerate=False)
    assert np.array_equal(host(th2.code), code) and np.array_equal(host(out2), host(out))
    it = dict(I=dI, I_low=dL, T_low=dT, s=s, k=k, T_hat=torch.empty((H, W, C), dtype=torch.float32, device="cuda"))
    plan = glu.BatchPlan([it], mode="exhaustive", degenerate=False)
    plan.launch()
    assert torch.equal(it["T_hat"], out2)
    plan.close()
    # the default candidate set reaches zero error where a pixel equals a
    # window colour; the pairs alone leave a residual there (unless k = 1 or
    # a single LR cell, where both take the lone cell)
    _, err_d = glu.search(dI, dL, s, k, 1e-3, "exhaustive", return_err=True)
    e_d = host(err_d)
    if k > 1 and L.shape[0] * L.shape[1] > 1:
        assert ((e_d == 0) & (e > 0)).any()
    else:
        assert np.array_equal(e, e_d)


@pytest.mark.parametrize("H,W,s,k,C,dt", [(200, 264, 8, 3, 3, "f32"), (37, 53, 4, 5, 1, "f32"), (29, 31, 3, 3, 3, "f16"),
                                           (41, 39, 4, 7, 2, "f32"), (50, 70, 2, 3, 3, "f32"), (61, 75, 6, 3, 4, "f32")])
def test_gnu_mode(H, W, s, k, C, dt):
    """GNU (nearest window colour, weight 1) through search, apply, the fused
    pass and a batch plan."""
    glu = _glu()
    log_case(test="gnu", H=H, W=W, s=s, k=k, C=C, dt=dt)
    I, L, T = _inputs(H, W, s, seed=H + W + 5, n_cells=max(4, H * W // 400), n_dots=3, C=C)
    dtype = torch.float16 if dt == "f16" else torch.float32
    _run_and_check(glu, I, L, T, s, k, "gnu", dtype=dtype)
    npd = np.float16 if dt == "f16" else np.float32
    it = dict(I=dev(I.astype(npd)), I_low=dev(L.astype(npd)), T_low=dev(T.astype(npd)), s=s, k=k,
              T_hat=torch.empty((H, W, C), dtype=dtype, device="cuda"))
    plan = glu.BatchPlan([it], mode="gnu")
    plan.launch()
    out, _ = glu.search_apply(it["I"], it["I_low"], it["T_low"], s, k, mode="gnu")
    assert torch.equal(out, it["T_hat"])
    plan.close()


@pytest.mark.parametrize("mode", ["exhaustive", "fast"])
def test_fused_step_graph_replays(mode):
    """The fused step on the 512 x 512 box x4 image, captured three times
    into one hipGraph and replayed three times with eager work between the
    replays: every replay writes bitwise the eager Theta and T_hat (the
    launches hold no memset or allocation)."""
    glu = _glu()
    log_case(test="fused_step_graph", mode=mode)
    I, L, T = _inputs(512, 512, 4, seed=1, n_cells=64, n_dots=20, dot_px=(2, 4), down="box")
    dI, dL, dT = dev(I), dev(L.astype(np.float32)), dev(T.astype(np.float32))
    th = glu.empty_theta(512, 512)
    out = torch.empty((512, 512, 3), dtype=torch.float32, device="cuda")
    glu.search_apply(dI, dL, dT, 4, 3, 1e-3, mode, theta=th, out=out)
    ref = (host(out), host(th.code), host(th.alpha))
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(3):
            glu.search_apply(dI, dL, dT, 4, 3, 1e-3, mode, theta=th, out=out)
    for _ in range(3):
        out.zero_()
        th.code.zero_()
        th.alpha.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(host(out), ref[0])
        assert np.array_equal(host(th.code), ref[1]) and np.array_equal(host(th.alpha), ref[2])
