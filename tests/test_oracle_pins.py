"""Pins for the float64 oracle: checks against what the paper and the
mathematics fix, independent of the oracle's own formulas.

Each test names the passage it pins.  None of these call the HIP library.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle as O
import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def _small_image(H, W, seed, n_cells=6, n_dots=2):
    return synth.voronoi(H, W, n_cells=n_cells, n_dots=n_dots, dot_px=(1, 2), sigma=0.01, seed=seed)


# ---------------------------------------------------------------------------
# Paper constants (Sec. 3.1, Sec. 3.2, Sec. 5.2)
# ---------------------------------------------------------------------------
def test_paper_parameters():
    g = _gold("paper_parameters.json")
    assert O.EPS == g["eps"]["value"]
    assert O.WINDOW == g["window"]["value"]
    assert O.TAU == pytest.approx(g["tau"]["value"], abs=1e-15)
    assert O.N_ITER == g["n_iter"]["value"]
    # A full 3x3 window holds 9 cells: 36 unordered pairs (Sec. 3.2), and
    # Algorithm 1 checks one pair per cell with the anchor fixed: 9.
    cells = O.window_cells(5, 5, 11, 11, 3)
    assert len(cells) == 9
    assert len(cells) * (len(cells) - 1) // 2 == g["pairs_3x3_exhaustive"]["value"]
    assert len(cells) == g["pairs_3x3_alg1"]["value"]


# ---------------------------------------------------------------------------
# Worked example on a colour segment (Eq. 4, Eq. 5), closed form
# ---------------------------------------------------------------------------
def _segment_setup(Ip):
    # HR 2 x 4, s = 2 -> LR 1 x 2: the window of pixel (0, 0) holds just the
    # two LR cells, L_a at index 0 and L_b at index 1.
    g = _gold("segment_example.json")
    L = np.array([[g["L_a"], g["L_b"]]], dtype=np.float64)
    I = np.full((2, 4, 3), 0.5)
    I[0, 0] = Ip
    return I, L


def test_segment_example_fixture_is_its_closed_form():
    """The stored worked example is what the committed generator writes from
    the closed forms of Eq. 4 and Eq. 5 (40-digit decimal arithmetic)."""
    import decimal
    import importlib.util

    spec = importlib.util.spec_from_file_location("make_segment_example",
                                                  os.path.join(GOLD, "make_segment_example.py"))
    gen = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(gen)
    with open(os.path.join(GOLD, "segment_example.json")) as f:
        stored = json.load(f, parse_float=decimal.Decimal)
    assert stored == json.loads(gen.text(), parse_float=decimal.Decimal)


@pytest.mark.parametrize("eps_key", ["eps", "zero"])
def test_segment_example_exhaustive(eps_key):
    g = _gold("segment_example.json")
    eps = g["eps"] if eps_key == "eps" else 0.0
    I, L = _segment_setup(g["I_p"])
    r = O.search_exhaustive(I, L, 2, 3, eps, pixels=[0])
    assert (int(r.a[0]), int(r.b[0])) == (0, 1)
    if eps_key == "eps":
        assert r.alpha[0] == pytest.approx(g["eq4_alpha"], abs=1e-15)
        assert r.err[0] == pytest.approx(g["eq4_err"], abs=1e-15)
    else:
        assert r.alpha[0] == pytest.approx(g["eps0_alpha"], abs=1e-15)
        assert r.err[0] == pytest.approx(0.0, abs=1e-15)


@pytest.mark.parametrize("eps_key", ["eps", "zero"])
def test_segment_example_fast(eps_key):
    g = _gold("segment_example.json")
    eps = g["eps"] if eps_key == "eps" else 0.0
    I, L = _segment_setup(g["I_p"])
    r = O.search_fast(I, L, 2, 3, eps, pixels=[0])
    assert (int(r.a[0]), int(r.b[0])) == (0, 1)  # anchor = nearest colour L_a
    if eps_key == "eps":
        assert r.alpha[0] == pytest.approx(g["eq5_alpha"], abs=1e-15)
        assert r.err[0] == pytest.approx(g["eq5_err"], abs=1e-15)
    else:
        assert r.alpha[0] == pytest.approx(g["eps0_alpha"], abs=1e-15)
        assert r.err[0] == pytest.approx(0.0, abs=1e-15)


def test_segment_orientation_swapped():
    # Same segment with t = 0.25: the exhaustive pair is still (0, 1) with
    # alpha the weight on cell 0 (Eq. 4: t l^2 / (l^2 + eps)); the fast anchor
    # moves to L_b (cell 1) because it is now the nearest colour.
    l2, eps, t = 2.0, 1e-3, 0.25
    I, L = _segment_setup([t, 0.0, 1.0 - t])
    r = O.search_exhaustive(I, L, 2, 3, eps, pixels=[0])
    assert (int(r.a[0]), int(r.b[0])) == (0, 1)
    assert r.alpha[0] == pytest.approx(t * l2 / (l2 + eps), abs=1e-15)
    f = O.search_fast(I, L, 2, 3, eps, pixels=[0])
    assert (int(f.a[0]), int(f.b[0])) == (1, 0)
    l = math.sqrt(l2)
    assert f.alpha[0] == pytest.approx((1 - t) * l / (l + eps), abs=1e-15)


# ---------------------------------------------------------------------------
# Brute force on tiny inputs: an independent minimisation over the segment
# ---------------------------------------------------------------------------
def _segment_min_bruteforce(Ip, Li, Lj):
    """min over t in [0, 1] of ||t Li + (1 - t) Lj - Ip||: dense grid + bounded scalar search."""
    from scipy.optimize import minimize_scalar

    f = lambda t: float(np.linalg.norm(t * Li + (1 - t) * Lj - Ip))
    ts = np.linspace(0.0, 1.0, 10001)
    vals = np.linalg.norm(ts[:, None] * Li[None] + (1 - ts)[:, None] * Lj[None] - Ip[None], axis=1)
    t0 = ts[int(np.argmin(vals))]
    lo, hi = max(0.0, t0 - 2e-4), min(1.0, t0 + 2e-4)
    res = minimize_scalar(f, bounds=(lo, hi), method="bounded", options={"xatol": 1e-13})
    cands = [(f(0.0), 0.0), (f(1.0), 1.0), (float(res.fun), float(res.x))]
    return min(cands)


@pytest.mark.parametrize("seed,H,W,s", [(11, 7, 9, 3), (12, 8, 8, 4), (13, 5, 11, 2), (14, 6, 6, 6), (15, 9, 4, 2)])
def test_exhaustive_bruteforce_eps0(seed, H, W, s):
    I = _small_image(H, W, seed)
    L = O.downsample_point(I, s)
    h, w = L.shape[:2]
    Lf = L.reshape(-1, 3).astype(np.float64)
    r = O.search_exhaustive(I, L, s, 3, 0.0)
    for p in range(H * W):
        y, x = divmod(p, W)
        Ip = I[y, x].astype(np.float64)
        cells = O.window_cells(y // s, x // s, h, w, 3)
        # the independent minimum over every unordered pair of the window
        best = min(
            _segment_min_bruteforce(Ip, Lf[ci], Lf[cj])[0]
            for ii, ci in enumerate(cells)
            for cj in cells[ii:]
        )
        assert r.err[p] == pytest.approx(best, abs=1e-9), p
        # the chosen pair lies in the window, is ordered, and attains its err
        a, b = int(r.a[p]), int(r.b[p])
        assert a in cells and b in cells and a <= b
        seg_best, t = _segment_min_bruteforce(Ip, Lf[a], Lf[b])
        assert seg_best == pytest.approx(r.err[p], abs=1e-9)
        if a != b and np.linalg.norm(Lf[a] - Lf[b]) > 1e-3:
            assert r.alpha[p] == pytest.approx(t, abs=1e-5)


@pytest.mark.parametrize("seed", [21, 22, 23])
def test_fast_bruteforce(seed):
    """Alg. 1 pinned by direct enumeration: a = nearest colour, b the best partner."""
    H, W, s, eps = 8, 10, 3, 1e-3
    I = _small_image(H, W, seed)
    L = O.downsample_point(I, s)
    h, w = L.shape[:2]
    Lf = L.reshape(-1, 3).astype(np.float64)
    r = O.search_fast(I, L, s, 3, eps)
    for p in range(H * W):
        y, x = divmod(p, W)
        Ip = I[y, x].astype(np.float64)
        cells = O.window_cells(y // s, x // s, h, w, 3)
        dists = [float(np.linalg.norm(Ip - Lf[c])) for c in cells]
        a = cells[int(np.argmin(dists))]
        assert int(r.a[p]) == a
        da = min(dists)
        errs = []
        for c, db in zip(cells, dists):
            om = 1.0 if c == a else db / (da + db + eps)
            errs.append((float(np.linalg.norm(om * Lf[a] + (1 - om) * Lf[c] - Ip)), c, om))
        e, c, om = min(errs, key=lambda v: v[0])
        assert r.err[p] == pytest.approx(e, abs=1e-12)
        # the fast weight lies in [0, 1] (Sec. 3.2)
        assert 0.0 <= r.alpha[p] <= 1.0


# ---------------------------------------------------------------------------
# Invariants
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("mode", ["exhaustive", "fast"])
@pytest.mark.parametrize("s,H,W", [(4, 16, 20), (3, 9, 12), (2, 7, 5)])
def test_nearest_copy_gives_zero_error(mode, s, H, W):
    """HR made of s x s replicas of LR: every pixel equals a window cell, so E = 0
    exactly and T_hat is nearest-neighbour upsampling of T_low."""
    rng = np.random.default_rng(s * 100 + H)
    h, w = O.lr_shape(H, W, s)
    L = rng.uniform(0, 1, (h, w, 3))
    I = np.repeat(np.repeat(L, s, 0), s, 1)[:H, :W]
    r = O.search(I, L, s, 3, O.EPS, mode)
    assert np.all(r.err == 0.0)
    T = rng.uniform(0, 1, (h, w, 2))
    That = O.apply(r.a, r.b, r.alpha, T).reshape(H, W, 2)
    nn = np.repeat(np.repeat(T, s, 0), s, 1)[:H, :W]
    np.testing.assert_allclose(That, nn, atol=0, rtol=0)


@pytest.mark.parametrize("mode", ["exhaustive", "fast"])
def test_constant_image(mode):
    c = np.array([0.3, 0.6, 0.2])
    I = np.broadcast_to(c, (12, 10, 3)).copy()
    L = O.downsample_point(I, 4)
    r = O.search(I, L, 4, 3, O.EPS, mode)
    assert np.all(r.err == 0.0)
    T = np.broadcast_to(np.array([0.7]), L.shape[:2] + (1,)).copy()
    That = O.apply(r.a, r.b, r.alpha, T)
    assert np.all(That == 0.7)


@pytest.mark.parametrize("mode", ["exhaustive", "fast"])
def test_alpha_range_and_gnu_bound(mode):
    """alpha in [0, 1]; GLU error <= GNU error (omega = 1, Sec. 3.2)."""
    I = _small_image(24, 28, 31, n_cells=10, n_dots=3)
    s = 4
    L = O.downsample_point(I, s)
    h, w = L.shape[:2]
    r = O.search(I, L, s, 3, O.EPS, mode)
    assert np.all((r.alpha >= 0) & (r.alpha <= 1))
    Lf = L.reshape(-1, 3).astype(np.float64)
    for p in range(0, 24 * 28, 7):
        y, x = divmod(p, 28)
        cells = O.window_cells(y // s, x // s, h, w, 3)
        gnu = min(np.linalg.norm(I[y, x].astype(np.float64) - Lf[c]) for c in cells)
        assert r.err[p] <= gnu + 1e-15


def test_exhaustive_not_worse_than_fast_eps0():
    I = _small_image(20, 24, 41, n_cells=8)
    L = O.downsample_point(I, 4)
    ex = O.search_exhaustive(I, L, 4, 3, 0.0)
    fa = O.search_fast(I, L, 4, 3, 0.0)
    assert np.all(ex.err <= fa.err + 1e-12)


def test_window_one_is_guided_nearest():
    """k = 1: Omega = {p_down}, so T_hat = T_low[p_down]."""
    I = _small_image(13, 17, 51)
    s = 4
    L = O.downsample_point(I, s)
    h, w = L.shape[:2]
    for mode in ("exhaustive", "fast"):
        r = O.search(I, L, s, 1, O.EPS, mode)
        ys, xs = np.divmod(np.arange(13 * 17), 17)
        cell = (ys // s) * w + xs // s
        assert np.all(r.a == cell) and np.all(r.b == cell)
        T = np.random.default_rng(0).uniform(0, 1, (h, w, 3))
        np.testing.assert_array_equal(O.apply(r.a, r.b, r.alpha, T), T.reshape(-1, 3)[cell])


def test_affine_transfer_and_self_reconstruction():
    """Sec. 4.1: if T_low = A I_low + t locally, the same Theta transfers it.
    Also apply(Theta, I_low) reproduces I_hat with ||I_hat - I|| = E."""
    I = _small_image(20, 20, 61, n_cells=7)
    s = 4
    L = O.downsample_point(I, s)
    r = O.search_exhaustive(I, L, s)
    rng = np.random.default_rng(1)
    A = rng.normal(size=(3, 3))
    t = rng.normal(size=3)
    TL = np.einsum("ij,hwj->hwi", A, L.astype(np.float64)) + t
    lhs = O.apply(r.a, r.b, r.alpha, TL)
    rhs = np.einsum("ij,nj->ni", A, O.apply(r.a, r.b, r.alpha, L)) + t
    np.testing.assert_allclose(lhs, rhs, atol=1e-12)
    Ihat = O.reconstruct(r.a, r.b, r.alpha, L)
    np.testing.assert_allclose(
        np.linalg.norm(Ihat - I.reshape(-1, 3).astype(np.float64), axis=1), r.err, atol=1e-12
    )


@pytest.mark.parametrize("mode", ["exhaustive", "fast"])
def test_channel_permutation_invariance(mode):
    I = _small_image(16, 20, 71)
    L = O.downsample_point(I, 4)
    perm = [2, 0, 1]
    r1 = O.search(I, L, 4, 3, O.EPS, mode)
    r2 = O.search(I[..., perm], L[..., perm], 4, 3, O.EPS, mode)
    np.testing.assert_array_equal(r1.a, r2.a)
    np.testing.assert_array_equal(r1.b, r2.b)
    np.testing.assert_allclose(r1.alpha, r2.alpha, atol=1e-12)


@pytest.mark.parametrize("mode", ["exhaustive", "fast"])
def test_transpose_symmetry(mode):
    """Transposing a square image (H, W multiples of s) transposes the errors.

    Eq. 4 with eps > 0 is not symmetric in (a, b): it shrinks the weight
    towards b, and transposing reorders the LR cells and so swaps the roles
    of some pairs.  The exhaustive check therefore uses eps = 0, where the
    weight is the exact segment projection; the fast weight (Eq. 5) and its
    anchor do not depend on the cell order."""
    I = _small_image(24, 24, 81, n_cells=9)
    s = 4
    eps = 0.0 if mode == "exhaustive" else O.EPS
    L = O.downsample_point(I, s)
    r1 = O.search(I, L, s, 3, eps, mode)
    r2 = O.search(I.transpose(1, 0, 2), L.transpose(1, 0, 2), s, 3, eps, mode)
    np.testing.assert_allclose(r1.err.reshape(24, 24), r2.err.reshape(24, 24).T, atol=1e-12)


def test_degenerate_reading():
    """With only the literal i < j pairs (36 for 3 x 3), a pixel equal to the
    first cell of its window keeps a residual error sqrt(n) eps / (n + eps);
    with the degenerate candidates it is 0."""
    L = np.zeros((3, 3, 3))
    L[..., 0] = np.arange(9).reshape(3, 3) / 8.0
    L[..., 1] = 0.5
    I = np.repeat(np.repeat(L, 2, 0), 2, 1)
    p = 0  # pixel (0, 0) equals L[0, 0], the first cell of its window
    lit = O.search_exhaustive(I, L, 2, 3, O.EPS, pixels=[p], degenerate=False)
    full = O.search_exhaustive(I, L, 2, 3, O.EPS, pixels=[p])
    assert full.err[0] == 0.0
    assert lit.err[0] > 0.0
    # closed form for the best literal pair (0, j): err = sqrt(n) eps / (n + eps)
    cells = O.window_cells(0, 0, 3, 3, 3)
    Lf = L.reshape(-1, 3)
    cf = min(math.sqrt(n) * O.EPS / (n + O.EPS) for n in (float(((Lf[0] - Lf[c]) ** 2).sum()) for c in cells[1:]))
    assert lit.err[0] == pytest.approx(cf, rel=1e-12)


# ---------------------------------------------------------------------------
# Downsampling
# ---------------------------------------------------------------------------
def test_downsample_point_and_box():
    I = np.arange(5 * 7 * 3, dtype=np.float64).reshape(5, 7, 3)
    p = O.downsample_point(I, 3)
    assert p.shape == (2, 3, 3)
    # offset floor(3/2) = 1, clamped into the image
    assert np.array_equal(p[0, 0], I[1, 1]) and np.array_equal(p[1, 2], I[4, 6])
    b = O.downsample_box(I, 3)
    np.testing.assert_allclose(b[1, 2], I[3:5, 6:7].reshape(-1, 3).mean(0))
    np.testing.assert_allclose(b[0, 0], I[0:3, 0:3].reshape(-1, 3).mean(0))


# ---------------------------------------------------------------------------
# Backward of Eq. 1
# ---------------------------------------------------------------------------
def _theta_small(seed=91, H=12, W=16, s=4, C=3):
    I = _small_image(H, W, seed)
    L = O.downsample_point(I, s)
    r = O.search_exhaustive(I, L, s)
    rng = np.random.default_rng(seed)
    T = rng.uniform(0, 1, L.shape[:2] + (C,))
    return r, T, rng


def test_backward_finite_differences():
    r, T, rng = _theta_small()
    target = rng.uniform(0, 1, (r.a.size, 3))

    def loss(alpha, T):
        return float(((O.apply(r.a, r.b, alpha, T) - target) ** 2).sum())

    out = O.apply(r.a, r.b, r.alpha, T)
    G = 2 * (out - target)
    da, dT = O.apply_backward(r.a, r.b, r.alpha, T, G)
    h = 1e-6
    for idx in rng.choice(T.size, 12, replace=False):
        Tp = T.copy().ravel()
        Tm = T.copy().ravel()
        Tp[idx] += h
        Tm[idx] -= h
        fd = (loss(r.alpha, Tp.reshape(T.shape)) - loss(r.alpha, Tm.reshape(T.shape))) / (2 * h)
        assert dT.ravel()[idx] == pytest.approx(fd, rel=1e-6, abs=1e-7)
    for p in rng.choice(r.a.size, 12, replace=False):
        ap = r.alpha.copy()
        am = r.alpha.copy()
        ap[p] += h
        am[p] -= h
        fd = (loss(ap, T) - loss(am, T)) / (2 * h)
        assert da[p] == pytest.approx(fd, rel=1e-6, abs=1e-7)


def test_backward_adjoint_and_torch_autograd():
    import torch

    r, T, rng = _theta_small(seed=92, C=2)
    # adjoint identity <apply(X), Y> = <X, apply^T(Y)> for the T_low slot
    X = rng.normal(size=T.shape)
    Y = rng.normal(size=(r.a.size, 2))
    lhs = float((O.apply(r.a, r.b, r.alpha, X) * Y).sum())
    _, dX = O.apply_backward(r.a, r.b, r.alpha, X, Y)
    rhs = float((X * dX).sum())
    assert lhs == pytest.approx(rhs, rel=1e-12)
    # float64 torch autograd reference built from index_select
    Tt = torch.tensor(T.reshape(-1, 2), dtype=torch.float64, requires_grad=True)
    at = torch.tensor(r.alpha, dtype=torch.float64, requires_grad=True)
    ia = torch.tensor(r.a)
    ib = torch.tensor(r.b)
    out = at[:, None] * Tt.index_select(0, ia) + (1 - at[:, None]) * Tt.index_select(0, ib)
    Gt = torch.tensor(Y)
    (out * Gt).sum().backward()
    da, dT = O.apply_backward(r.a, r.b, r.alpha, T, Y)
    np.testing.assert_allclose(at.grad.numpy(), da, atol=1e-12)
    np.testing.assert_allclose(Tt.grad.numpy().reshape(T.shape), dT, atol=1e-12)


# ---------------------------------------------------------------------------
# Connected components and Algorithm 2
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_ccl8_matches_scipy(seed):
    from scipy import ndimage

    rng = np.random.default_rng(seed)
    mask = rng.uniform(size=(37, 41)) < 0.35
    lab, M = O.ccl8(mask)
    ref, Mr = ndimage.label(mask, structure=np.ones((3, 3)))
    assert M == Mr
    np.testing.assert_array_equal(lab, ref)


def _dot_image(H=64, W=64, s=8, dot=(17, 41), size=2, bg=(0.4, 0.5, 0.6), col=(0.95, 0.1, 0.1)):
    I = np.empty((H, W, 3))
    I[:] = bg
    y, x = dot
    I[y : y + size, x : x + size] = col
    return I


def test_joint_recovers_missed_dot():
    """Sec. 3.3: a small isolated dot that regular-grid sampling misses is added
    to I_down in one round, its pixels drop below tau, and the trial is accepted."""
    s = 8
    I = _dot_image()
    L0 = O.downsample_point(I, s)
    assert not np.any(np.all(L0 == np.array([0.95, 0.1, 0.1]), axis=-1))
    res = O.joint_downsample(I, L0, s, tau=O.TAU, max_iter=3)
    assert res.n_components[0] == 1 and res.n_accepted[0] == 1
    assert np.any(np.all(res.L == np.array([0.95, 0.1, 0.1]), axis=-1))
    dot_pixels = [17 * 64 + 41, 17 * 64 + 42, 18 * 64 + 41, 18 * 64 + 42]
    assert np.all(res.err[dot_pixels] < O.TAU)
    assert res.rounds_run == 1  # round 2 finds no large error and stops
    assert res.err_sum_final < res.err_sum_initial


def test_joint_invariants_on_voronoi():
    s = 8
    I = synth.voronoi(96, 120, n_cells=20, n_dots=10, dot_px=(1, 3), seed=7)
    L0 = O.downsample_point(I, s)
    res = O.joint_downsample(I, L0, s, tau=O.TAU, max_iter=3)
    # the sum of errors never increases over accepted trials
    assert res.err_sum_final <= res.err_sum_initial
    for d in res.log:
        if d.accepted:
            assert d.e1 <= d.e0
    # the final Theta is the search on the final I_down (a fixpoint)
    again = O.search_exhaustive(I, res.L, s)
    np.testing.assert_array_equal(again.a, res.a)
    np.testing.assert_array_equal(again.b, res.b)
    np.testing.assert_allclose(again.err, res.err, atol=0)
    # every LR pixel is its initial value or a copy of an HR pixel of its block
    h, w = L0.shape[:2]
    for qy in range(h):
        for qx in range(w):
            v = res.L[qy, qx]
            if np.array_equal(v, L0[qy, qx]):
                continue
            blk = I[qy * s : qy * s + s, qx * s : qx * s + s].reshape(-1, 3).astype(np.float64)
            assert np.any(np.all(blk == v, axis=1))


def test_joint_no_large_error_is_a_no_op():
    s = 4
    rng = np.random.default_rng(3)
    L = rng.uniform(0, 1, (5, 6, 3))
    I = np.repeat(np.repeat(L, s, 0), s, 1)
    res = O.joint_downsample(I, L, s)
    assert res.rounds_run == 0 and res.log == []
    np.testing.assert_array_equal(res.L, L)


def test_joint_constructed_rollback():
    """Direct construction of a rejected trial (Alg. 2 rollback, e1 > e0).

    A 2 x 2 dot of colour Z sits in the middle block, whose regular-grid
    sample is the only LR pixel of colour X; every other sample is Y.
    Replacing that sample with Z fixes the 4 dot pixels (each 0.653 away from
    segment XY) but leaves the other 60 pixels of the block 0.588 away from
    segment YZ, so the total error rises and the trial is rolled back."""
    s = 8
    H = W = 24
    X, Y, Z = (0.2, 0.2, 0.2), (0.6, 0.6, 0.6), (0.9, 0.1, 0.1)
    I = np.empty((H, W, 3))
    I[:] = Y
    I[8:16, 8:16] = X
    I[9:11, 9:11] = Z
    L0 = O.downsample_point(I, s)
    res = O.joint_downsample(I, L0, s, tau=O.TAU, max_iter=1)
    assert len(res.log) == 1
    d = res.log[0]
    assert d.q_pstar == [(4, 9 * W + 9)]
    assert not d.accepted and d.e1 > d.e0
    np.testing.assert_array_equal(res.L, L0)


def test_joint_literal_reading_sums_the_component():
    """The literal reading of Alg. 2 re-searches and sums E over the
    component alone.  On the constructed rollback image (a 2 x 2 dot Z inside
    the block whose sample X is replaced) the two readings decide apart: the
    dot's own error falls from 4 times its distance to segment XY to exactly 0
    (each dot pixel now equals an LR colour), so the literal trial is kept,
    while the affected set also counts the 60 other pixels of the block,
    which end 0.588 away from segment YZ, and rolls back.  The kept literal
    trial leaves those 60 pixels' Theta and E as they were (stale), unlike a
    fresh search on the final I_down."""
    s = 8
    H = W = 24
    X, Y, Z = (0.2, 0.2, 0.2), (0.6, 0.6, 0.6), (0.9, 0.1, 0.1)
    I = np.empty((H, W, 3))
    I[:] = Y
    I[8:16, 8:16] = X
    I[9:11, 9:11] = Z
    L0 = O.downsample_point(I, s)
    dot = np.array([9 * W + 9, 9 * W + 10, 10 * W + 9, 10 * W + 10])
    init = O.search_exhaustive(I, L0, s)
    lit = O.joint_downsample(I, L0, s, tau=O.TAU, max_iter=1, reading="literal")
    aff = O.joint_downsample(I, L0, s, tau=O.TAU, max_iter=1)
    assert len(lit.log) == 1 and len(aff.log) == 1
    d = lit.log[0]
    assert d.accepted and not aff.log[0].accepted
    assert d.q_pstar == [(4, 9 * W + 9)]
    assert d.e0 == pytest.approx(float(init.err[dot].sum()), abs=1e-15)
    assert d.e0 > 4 * 0.6
    assert d.e1 == 0.0
    assert np.array_equal(lit.L[1, 1], np.array(Z))
    # pixels of the block outside the component keep their initial (stale) E
    blk = np.zeros((H, W), dtype=bool)
    blk[8:16, 8:16] = True
    blk.ravel()[dot] = False
    rest = np.flatnonzero(blk)
    np.testing.assert_array_equal(lit.err[rest], init.err[rest])
    fresh = O.search_exhaustive(I, lit.L, s)
    assert np.all(fresh.err[rest] > 0.5)
    assert lit.err_sum_final < lit.err_sum_initial < float(fresh.err.sum())


# ---------------------------------------------------------------------------
# Pair evaluators used to check another implementation's choice
# ---------------------------------------------------------------------------
def test_pair_evaluators_reproduce_search():
    """Evaluating the search's own winners gives back its weight and error,
    and the fast search with its own anchor given is the fast search."""
    I = _small_image(30, 36, 101, n_cells=8, n_dots=3)
    s = 4
    L = O.downsample_point(I, s)
    pix = np.arange(30 * 36)
    ex = O.search_exhaustive(I, L, s)
    al, e = O.eval_pairs_exhaustive(I, L, pix, ex.a, ex.b)
    np.testing.assert_allclose(al, ex.alpha, atol=1e-15)
    np.testing.assert_allclose(e, ex.err, atol=1e-15)
    fa = O.search_fast(I, L, s)
    om, e2 = O.eval_pairs_fast(I, L, pix, fa.a, fa.b)
    np.testing.assert_allclose(om, fa.alpha, atol=1e-15)
    np.testing.assert_allclose(e2, fa.err, atol=1e-15)
    g = O.search_fast_given_anchor(I, L, s, 3, O.EPS, pix, fa.a)
    np.testing.assert_array_equal(g.b, fa.b)
    np.testing.assert_allclose(g.err, fa.err, atol=1e-15)
    # with another anchor the error can only grow or stay (b = a is allowed)
    other = np.where(fa.a == ex.a, ex.b, ex.a)
    g2 = O.search_fast_given_anchor(I, L, s, 3, O.EPS, pix, other)
    d_other = np.linalg.norm(I.reshape(-1, 3).astype(np.float64) - L.reshape(-1, 3)[other], axis=1)
    assert np.all(g2.err <= d_other + 1e-15)


def test_exact_ties_go_to_the_earliest_candidate():
    """Reading of the tie rule: the first candidate in colexicographic order
    wins an exact tie (exhaustive), and the anchor is the first cell of least
    distance (fast).  Cells 0 and 4 of the window carry the same colour, equal
    to the pixel: (0, 0) comes before every other zero-error candidate."""
    L = np.zeros((3, 3, 3))
    L[..., 0] = np.arange(9).reshape(3, 3) / 9.0
    L[..., 1] = 0.3
    L[1, 1] = L[0, 0]
    I = np.repeat(np.repeat(L, 2, 0), 2, 1)
    p = 1 * 6 + 2  # pixel (1, 2): its window is the whole 3 x 3 LR image, centre cell 4
    I[1, 2] = L[0, 0]
    ex = O.search_exhaustive(I, L, 2, 3, O.EPS, pixels=[p])
    assert (int(ex.a[0]), int(ex.b[0])) == (0, 0) and ex.err[0] == 0.0
    fa = O.search_fast(I, L, 2, 3, O.EPS, pixels=[p])
    assert int(fa.a[0]) == 0 and int(fa.b[0]) == 0


def test_joint_replacement_takes_the_largest_error():
    """Alg. 2 replaces I_down[q] by the pixel of [q_up] & C with the largest
    error: a two-colour dot whose brighter pixel is farther from the
    background puts that colour into I_down."""
    s = 8
    I = np.empty((64, 64, 3))
    I[:] = (0.4, 0.5, 0.6)
    far, near = (0.95, 0.05, 0.05), (0.75, 0.35, 0.35)
    # off the block's sampling point (20, 20), so neither colour is in I_down
    I[18, 18] = near
    I[18, 19] = far
    L0 = O.downsample_point(I, s)
    res = O.joint_downsample(I, L0, s, tau=O.TAU, max_iter=1)
    d = res.log[0]
    assert d.q_pstar == [(2 * 8 + 2, 18 * 64 + 19)]
    assert np.array_equal(res.L[2, 2], np.array(far))


# --------------------------------------------------------------------------
# Gradient-driven joint downsampling (defined by the project, not the paper)
# --------------------------------------------------------------------------
def test_self_upsampling_gradient_finite_differences():
    """D equals central finite differences of sum_p ||apply(Theta, L) - I||^2
    with Theta fixed (the loss is quadratic in L, so central differences are
    exact up to rounding)."""
    s = 4
    I = synth.voronoi(12, 16, n_cells=5, n_dots=1, dot_px=(1, 2), seed=11).astype(np.float64)
    L = O.downsample_point(I, s) + 0.05 * np.random.default_rng(2).standard_normal((3, 4, 3))
    r = O.search_exhaustive(I, L, s)
    D, I_hat = O.self_upsampling_gradient(I, L, r.a, r.b, r.alpha)

    def loss(Lx):
        return float(((O.apply(r.a, r.b, r.alpha, Lx).reshape(I.shape) - I) ** 2).sum())

    h = 1e-6
    fd = np.zeros_like(L)
    for idx in np.ndindex(L.shape):
        Lp, Lm = L.copy(), L.copy()
        Lp[idx] += h
        Lm[idx] -= h
        fd[idx] = (loss(Lp) - loss(Lm)) / (2 * h)
    np.testing.assert_allclose(D, fd, rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(I_hat.reshape(-1, 3), O.apply(r.a, r.b, r.alpha, L), atol=0)


def test_snap_to_block_bruteforce():
    """The nearest pixel of each block, by an independent double loop over all
    HR pixels (first minimum in raster order), including ragged border blocks
    and exact ties."""
    rng = np.random.default_rng(5)
    H, W, s = 11, 13, 4
    I = rng.integers(0, 4, (H, W, 3)) / 4.0  # coarse colours: many exact ties
    Z = rng.uniform(0, 1, (3, 4, 3))
    # in every other block, Z is the colour of a pixel that recurs later in the block
    for qy in range(3):
        for qx in range(0, 4, 2):
            y0, x0 = qy * s, qx * s
            y1, x1 = min(H, y0 + s) - 1, min(W, x0 + s) - 1
            I[y1, x1] = I[y0, x0 + 1]
            Z[qy, qx] = I[y0, x0 + 1]
    # and in block (0, 1) the nearest pixel is the only one of its colour, in
    # the block's last column
    I[1, 2 * s - 1] = (0.9, 0.9, 0.9)
    Z[0, 1] = (0.88, 0.9, 0.91)
    got = O.snap_to_block(I, Z, s)
    for qy in range(3):
        for qx in range(4):
            best, arg = None, None
            for y in range(H):
                for x in range(W):
                    if y // s != qy or x // s != qx:
                        continue
                    d = sum((float(I[y, x, c]) - float(Z[qy, qx, c])) ** 2 for c in range(3))
                    if best is None or d < best:
                        best, arg = d, y * W + x
            assert got[qy * 4 + qx] == arg


def test_gradient_joint_fixed_points():
    """eta = 0 keeps a regular-grid I_down (each L_q is a pixel of its block, at
    distance 0); a nearest-neighbour copy image has E = 0 and zero gradient."""
    s = 4
    I = synth.voronoi(24, 32, n_cells=6, n_dots=2, dot_px=(1, 2), seed=3).astype(np.float64)
    L0 = O.downsample_point(I, s)
    r = O.joint_downsample_gradient(I, L0, s, eta=0.0, n_steps=2, keep_best=False)
    np.testing.assert_array_equal(r.L, L0)
    assert r.err_sums[0] == r.err_sums[1] == r.err_sums[2]
    Lc = np.random.default_rng(4).uniform(0, 1, (6, 8, 3))
    Inn = np.repeat(np.repeat(Lc, s, axis=0), s, axis=1)
    r = O.joint_downsample_gradient(Inn, Lc, s, eta=0.05, n_steps=2, keep_best=False)
    np.testing.assert_array_equal(r.L, Lc)
    assert max(r.err_sums) == 0.0


def test_gradient_joint_best_and_copies():
    """The returned I_down has the least sum of E seen (the first on ties), its
    Theta and E are the search on it, and every LR pixel is a copy of an HR
    pixel of its own block; on this image one step lowers the sum of E."""
    s = 8
    I = synth.voronoi(96, 120, n_cells=20, n_dots=10, dot_px=(1, 3), seed=7)
    L0 = O.downsample_point(I, s)
    r = O.joint_downsample_gradient(I, L0, s, eta=0.01, n_steps=3, keep_best=True)
    assert r.err_sums[1] < r.err_sums[0]
    assert float(r.err.sum()) == min(r.err_sums) == r.err_sums[r.best_step]
    assert r.best_step == int(np.argmin(r.err_sums))
    again = O.search_exhaustive(I, r.L, s)
    np.testing.assert_array_equal(again.a, r.a)
    np.testing.assert_array_equal(again.err, r.err)
    h, w = L0.shape[:2]
    If = I.astype(np.float64)
    for qy in range(h):
        for qx in range(w):
            blk = If[qy * s : qy * s + s, qx * s : qx * s + s].reshape(-1, 3)
            assert np.any(np.all(blk == r.L[qy, qx], axis=1))


def test_gnu_is_the_nearest_window_colour():
    """GNU (Sec. 3.2): per pixel the nearest colour of the truncated window by
    an independent double loop (first on ties), weight 1, err its distance;
    the GLU searches never do worse, and GNU's a is fast mode's anchor."""
    s, k = 4, 3
    I = synth.voronoi(20, 24, n_cells=6, n_dots=2, dot_px=(1, 2), seed=13).astype(np.float64)
    L = O.downsample_point(I, s)
    L[1, 2] = L[1, 1]  # an exact colour tie inside some windows
    g = O.search_gnu(I, L, s, k)
    H, W = I.shape[:2]
    h, w = L.shape[:2]
    for y in range(H):
        for x in range(W):
            best, arg = None, None
            for cy in range(max(0, y // s - 1), min(h, y // s + 2)):
                for cx in range(max(0, x // s - 1), min(w, x // s + 2)):
                    dd = math.sqrt(sum((I[y, x, c] - L[cy, cx, c]) ** 2 for c in range(3)))
                    if best is None or dd < best:
                        best, arg = dd, cy * w + cx
            p = y * W + x
            assert g.a[p] == arg and g.b[p] == arg and g.alpha[p] == 1.0
            assert abs(g.err[p] - best) <= 1e-12
    ex = O.search_exhaustive(I, L, s, k)
    fa = O.search_fast(I, L, s, k)
    assert np.all(ex.err <= g.err + 1e-12) and np.all(fa.err <= g.err + 1e-12)
    np.testing.assert_array_equal(fa.a, g.a)
    # GNU upsampling copies the target of the anchor cell
    T = np.random.default_rng(1).uniform(0, 1, (h, w, 2))
    np.testing.assert_array_equal(O.apply(g.a, g.b, g.alpha, T), T.reshape(-1, 2)[g.a])
