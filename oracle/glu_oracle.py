"""Plain float64 CPU oracle for guided linear upsampling (GLU).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or
links this module: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it, to check the HIP kernels and to
time a CPU reference.  It shares no code with the HIP path.

Written from the paper (Song et al., "Guided Linear Upsampling", ACM TOG
42(4), 2023).  Each function computes the paper's definition directly (the
search, Eq. 1 and its gradient) or, for the heuristic of Alg. 2, takes its
steps in the paper's order; NumPy arrays run each step over many pixels at
once, but no step is blocked, fused or reordered.  All arithmetic is
float64: inputs that arrive as float32 or float16 are upcast exactly.

Notation (Sec. 3.1):
  I      high-resolution guide, H x W x 3
  L      low-resolution guide I_down, h x w x 3, h = ceil(H/s), w = ceil(W/s)
  p_down (y // s, x // s), the LR cell under HR pixel p
  Omega  the k x k LR cells centred on p_down, truncated at the LR border
  Theta  per pixel (a, b, alpha): LR linear indices of the two endpoints and
         the weight on a
  E      per-pixel error ||I_p - I_hat_p|| (Euclidean over RGB, not squared)

Readings of points the paper leaves open (each also listed in the design
notes of the repository):
  * alpha from the projection formula (Eq. 4) is clamped to [0, 1]: the
    model is an interpolation (Eq. 1) and the fast weight (Eq. 5) is in
    [0, 1] by construction.
  * The candidate set of the exhaustive search holds every unordered pair
    i < j of the window (36 for 3 x 3, Sec. 3.2) plus the degenerate pairs
    (i, i) with alpha = 1, which make nearest-neighbour upsampling (GNU,
    Sec. 3.2) a special case of the search.
  * Candidates are visited in colexicographic order of (i, j) in LR linear
    index (second index outer, first index inner, (j, j) after (i < j, j));
    the first strict minimum wins, so exact ties go to the earliest
    candidate in that order.  The fast search takes the anchor a as the
    first minimum of the colour distance and b as the first minimum of the
    error, both in ascending LR index.
  * If a denominator is zero (only possible with eps = 0) the weight is 1.
  * The same eps (default 1e-3, Sec. 3.1) is used in Eq. 4 and Eq. 5.
  * Joint downsampling (Alg. 2): 8-connected components, ordered by their
    first pixel in raster order, processed one after another; by default
    the pixels re-searched and summed for e0 / e1 are the whole affected
    set A = {p : Omega(p) meets Q}; ``reading="literal"`` re-searches and
    sums over the component only.  Rollback when e1 > e0 (strict).
    Arg-max ties go to the smallest HR linear index.
"""
from __future__ import annotations

import math
from collections import deque
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "EPS",
    "TAU",
    "N_ITER",
    "WINDOW",
    "lr_shape",
    "downsample_point",
    "downsample_box",
    "window_cells",
    "search_exhaustive",
    "search_fast",
    "search_gnu",
    "search",
    "apply",
    "apply_backward",
    "reconstruct",
    "ccl8",
    "joint_downsample",
    "JointResult",
    "eval_pairs_exhaustive",
    "eval_pairs_fast",
    "search_fast_given_anchor",
    "self_upsampling_gradient",
    "snap_to_block",
    "joint_downsample_gradient",
    "GradientJointResult",
]

# Parameters fixed by the paper: eps of Eq. 4 (Sec. 3.1); window S = 3,
# tau = 30/255 and N = 3 iterations (Sec. 5.2).
EPS = 1e-3
WINDOW = 3
TAU = 30.0 / 255.0
N_ITER = 3


def lr_shape(H: int, W: int, s: int) -> tuple[int, int]:
    """LR size for ratio s: every HR pixel has a cell, so ceil(H/s) x ceil(W/s)."""
    return (-(-H // s), -(-W // s))


# --------------------------------------------------------------------------
# Downsampling (inputs of the search)
# --------------------------------------------------------------------------
def downsample_point(I: np.ndarray, s: int) -> np.ndarray:
    """Regular-grid downsampling (Sec. 3.1, Alg. 2 initialisation).

    Each LR pixel is a copy of exactly one HR pixel (Sec. 3.3): the pixel at
    offset floor(s/2) inside its s x s block, clamped into the image.
    Returns an array of I's dtype (a copy of stored values, no rounding).
    """
    I = np.asarray(I)
    H, W = I.shape[:2]
    h, w = lr_shape(H, W, s)
    ys = np.minimum(np.arange(h) * s + s // 2, H - 1)
    xs = np.minimum(np.arange(w) * s + s // 2, W - 1)
    return np.ascontiguousarray(I[ys][:, xs])


def downsample_box(I: np.ndarray, s: int) -> np.ndarray:
    """Box downsampling: mean of the in-image pixels of each s x s block (float64)."""
    I = np.asarray(I, dtype=np.float64)
    H, W, C = I.shape
    h, w = lr_shape(H, W, s)
    out = np.zeros((h, w, C), dtype=np.float64)
    for qy in range(h):
        for qx in range(w):
            blk = I[qy * s : min(H, qy * s + s), qx * s : min(W, qx * s + s)]
            out[qy, qx] = blk.reshape(-1, C).mean(axis=0)
    return out


# --------------------------------------------------------------------------
# Windows
# --------------------------------------------------------------------------
def window_cells(qy: int, qx: int, h: int, w: int, k: int) -> list[int]:
    """LR linear indices of Omega around cell (qy, qx), ascending, border-truncated."""
    r = k // 2
    out = []
    for dy in range(-r, r + 1):
        for dx in range(-r, r + 1):
            y, x = qy + dy, qx + dx
            if 0 <= y < h and 0 <= x < w:
                out.append(y * w + x)
    return out


def _pixel_coords(H: int, W: int, pixels):
    if pixels is None:
        ys, xs = np.divmod(np.arange(H * W, dtype=np.int64), W)
    else:
        pixels = np.asarray(pixels, dtype=np.int64).ravel()
        ys, xs = np.divmod(pixels, W)
    return ys, xs


def _candidates(ys, xs, s, h, w, k):
    """Per window offset (ascending): validity mask and LR linear index per pixel."""
    r = k // 2
    qy = ys // s
    qx = xs // s
    out = []
    for dy in range(-r, r + 1):
        for dx in range(-r, r + 1):
            cy = qy + dy
            cx = qx + dx
            valid = (cy >= 0) & (cy < h) & (cx >= 0) & (cx < w)
            lin = np.where(valid, cy * w + cx, 0)
            out.append((valid, lin))
    return out


@dataclass
class SearchResult:
    a: np.ndarray  # LR linear index of endpoint a (weight alpha)
    b: np.ndarray  # LR linear index of endpoint b (weight 1 - alpha)
    alpha: np.ndarray
    err: np.ndarray  # ||alpha L_a + (1 - alpha) L_b - I_p||
    pixels: np.ndarray | None = None  # flat HR indices searched (None: all)


def search_exhaustive(I, L, s, k=WINDOW, eps=EPS, pixels=None, degenerate=True) -> SearchResult:
    """Per-pixel pair search over all pairs of the window (Eq. 3 with Eq. 4).

    For every candidate pair (i, j), i <= j, of Omega(p):
        alpha = 1                                   if i == j
        alpha = clamp(((I_p - L_j) . (L_i - L_j)) / (||L_i - L_j||^2 + eps), 0, 1)
                                                    otherwise (1 if the denominator is 0)
        err   = ||alpha L_i + (1 - alpha) L_j - I_p||
    and keep the pair with the least err (first in colexicographic order on
    exact ties).  ``pixels`` restricts the search to flat HR indices.
    ``degenerate=False`` drops the (i, i) candidates except in a window with
    a single cell (the paper's literal 36 pairs for 3 x 3).
    """
    I = np.asarray(I, dtype=np.float64)
    L = np.asarray(L, dtype=np.float64)
    H, W = I.shape[:2]
    h, w = L.shape[:2]
    if (h, w) != lr_shape(H, W, s):
        raise ValueError("I_low must be ceil(H/s) x ceil(W/s)")
    ys, xs = _pixel_coords(H, W, pixels)
    Ip = I[ys, xs]  # (n, 3)
    Lf = L.reshape(-1, L.shape[2])
    cand = _candidates(ys, xs, s, h, w, k)
    n = Ip.shape[0]
    best = np.full(n, np.inf)
    a = np.full(n, -1, dtype=np.int64)
    b = np.full(n, -1, dtype=np.int64)
    alpha = np.full(n, np.nan)
    cols = [Lf[lin] for (_, lin) in cand]
    K = len(cand)
    for j in range(K):  # colexicographic: second index outer
        vj, linj = cand[j]
        Lj = cols[j]
        for i in range(j + 1):
            vi, lini = cand[i]
            Li = cols[i]
            if i == j:
                if not degenerate:
                    continue
                al = np.ones(n)
            else:
                e = Li - Lj
                den = np.einsum("nc,nc->n", e, e) + eps
                g = np.einsum("nc,nc->n", Ip - Lj, e)
                with np.errstate(divide="ignore", invalid="ignore"):
                    al = np.where(den > 0, np.clip(g / np.where(den > 0, den, 1.0), 0.0, 1.0), 1.0)
            rec = al[:, None] * Li + (1.0 - al)[:, None] * Lj
            err = np.sqrt(np.einsum("nc,nc->n", rec - Ip, rec - Ip))
            upd = vi & vj & (err < best)
            best = np.where(upd, err, best)
            a = np.where(upd, lini, a)
            b = np.where(upd, linj, b)
            alpha = np.where(upd, al, alpha)
    if not degenerate:
        # A window with a single cell has no proper pair: use its only cell.
        lone = a < 0
        if lone.any():
            for j in range(K):
                vj, linj = cand[j]
                take = lone & vj
                d = Ip - cols[j]
                err = np.sqrt(np.einsum("nc,nc->n", d, d))
                a = np.where(take, linj, a)
                b = np.where(take, linj, b)
                alpha = np.where(take, 1.0, alpha)
                best = np.where(take, err, best)
                lone = lone & ~vj
    return SearchResult(a=a, b=b, alpha=alpha, err=best, pixels=None if pixels is None else np.asarray(pixels))


def search_fast(I, L, s, k=WINDOW, eps=EPS, pixels=None) -> SearchResult:
    """Efficient search of Algorithm 1 with the weight of Eq. 5.

    a = the window cell of most similar colour to I_p (least Euclidean
    distance; first in ascending LR index on ties).  Then, with a fixed, for
    each b of the window (b = a allowed, weight 1):
        w_b   = ||I_p - L_b|| / (||I_p - L_a|| + ||I_p - L_b|| + eps)
        err_b = ||w_b L_a + (1 - w_b) L_b - I_p||
    and keep the first b of least err.
    """
    I = np.asarray(I, dtype=np.float64)
    L = np.asarray(L, dtype=np.float64)
    H, W = I.shape[:2]
    h, w = L.shape[:2]
    if (h, w) != lr_shape(H, W, s):
        raise ValueError("I_low must be ceil(H/s) x ceil(W/s)")
    ys, xs = _pixel_coords(H, W, pixels)
    Ip = I[ys, xs]
    Lf = L.reshape(-1, L.shape[2])
    cand = _candidates(ys, xs, s, h, w, k)
    n = Ip.shape[0]
    cols = [Lf[lin] for (_, lin) in cand]
    dist = []
    for (v, _), Lc in zip(cand, cols):
        d = Ip - Lc
        dist.append(np.where(v, np.sqrt(np.einsum("nc,nc->n", d, d)), np.inf))
    # anchor
    da = np.full(n, np.inf)
    ia = np.full(n, -1, dtype=np.int64)
    for idx, dd in enumerate(dist):
        upd = dd < da
        da = np.where(upd, dd, da)
        ia = np.where(upd, idx, ia)
    rows = np.arange(n)
    lin_all = np.stack([lin for (_, lin) in cand], axis=1)
    col_all = np.stack(cols, axis=1)  # (n, K, 3)
    a = lin_all[rows, ia]
    La = col_all[rows, ia]
    best = np.full(n, np.inf)
    b = np.full(n, -1, dtype=np.int64)
    omega = np.full(n, np.nan)
    for idx, ((v, lin), Lb) in enumerate(zip(cand, cols)):
        same = ia == idx
        den = da + dist[idx] + eps
        with np.errstate(divide="ignore", invalid="ignore"):
            om = np.where(den > 0, dist[idx] / np.where(den > 0, den, 1.0), 1.0)
        om = np.where(same, 1.0, om)
        rec = om[:, None] * La + (1.0 - om)[:, None] * Lb
        err = np.sqrt(np.einsum("nc,nc->n", rec - Ip, rec - Ip))
        upd = v & (err < best)
        best = np.where(upd, err, best)
        b = np.where(upd, lin, b)
        omega = np.where(upd, om, omega)
    return SearchResult(a=a, b=b, alpha=omega, err=best, pixels=None if pixels is None else np.asarray(pixels))


def search_gnu(I, L, s, k=WINDOW, pixels=None) -> SearchResult:
    """Guided nearest-neighbour upsampling (GNU, Sec. 3.2), the omega = 1
    special case of the model: a = b = the window cell of least Euclidean
    colour distance to I_p (first in ascending LR index on ties), weight 1,
    err = that distance."""
    I = np.asarray(I, dtype=np.float64)
    L = np.asarray(L, dtype=np.float64)
    H, W = I.shape[:2]
    h, w = L.shape[:2]
    if (h, w) != lr_shape(H, W, s):
        raise ValueError("I_low must be ceil(H/s) x ceil(W/s)")
    ys, xs = _pixel_coords(H, W, pixels)
    Ip = I[ys, xs]
    Lf = L.reshape(-1, L.shape[2])
    n = Ip.shape[0]
    da = np.full(n, np.inf)
    a = np.full(n, -1, dtype=np.int64)
    for v, lin in _candidates(ys, xs, s, h, w, k):
        d = Ip - Lf[lin]
        dd = np.where(v, np.sqrt(np.einsum("nc,nc->n", d, d)), np.inf)
        upd = dd < da
        da = np.where(upd, dd, da)
        a = np.where(upd, lin, a)
    return SearchResult(a=a, b=a.copy(), alpha=np.ones(n), err=da, pixels=None if pixels is None else np.asarray(pixels))


def search(I, L, s, k=WINDOW, eps=EPS, mode="exhaustive", pixels=None) -> SearchResult:
    if mode == "exhaustive":
        return search_exhaustive(I, L, s, k, eps, pixels)
    if mode == "fast":
        return search_fast(I, L, s, k, eps, pixels)
    if mode == "gnu":
        return search_gnu(I, L, s, k, pixels)
    raise ValueError("mode must be 'exhaustive', 'fast' or 'gnu'")


# --------------------------------------------------------------------------
# Apply (Eq. 1) and its backward
# --------------------------------------------------------------------------
def apply(a, b, alpha, T_low) -> np.ndarray:
    """Eq. 1: T_hat_p = alpha T_low[a] + (1 - alpha) T_low[b], per channel.

    ``a``, ``b``, ``alpha`` have the HR shape (H, W) (or any shape); returns
    that shape plus the channel axis of ``T_low`` (h, w, C).
    """
    T = np.asarray(T_low, dtype=np.float64)
    Tf = T.reshape(-1, T.shape[-1])
    al = np.asarray(alpha, dtype=np.float64)[..., None]
    return al * Tf[np.asarray(a)] + (1.0 - al) * Tf[np.asarray(b)]


def reconstruct(a, b, alpha, L) -> np.ndarray:
    """I_hat: Eq. 1 applied to the LR guide itself (self-upsampling, Sec. 3.3)."""
    return apply(a, b, alpha, L)


def apply_backward(a, b, alpha, T_low, G):
    """Gradients of Eq. 1 with Theta held fixed.

    dL/dalpha_p  = sum_c G_p,c (T_low[a_p],c - T_low[b_p],c)
    dL/dT_low_q  = sum_{p: a_p = q} alpha_p G_p + sum_{p: b_p = q} (1 - alpha_p) G_p
    """
    T = np.asarray(T_low, dtype=np.float64)
    C = T.shape[-1]
    Tf = T.reshape(-1, C)
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    al = np.asarray(alpha, dtype=np.float64).ravel()
    Gf = np.asarray(G, dtype=np.float64).reshape(-1, C)
    d_alpha = np.einsum("nc,nc->n", Gf, Tf[a] - Tf[b])
    dT = np.zeros_like(Tf)
    np.add.at(dT, a, al[:, None] * Gf)
    np.add.at(dT, b, (1.0 - al)[:, None] * Gf)
    return d_alpha.reshape(np.shape(alpha)), dT.reshape(T.shape)


# --------------------------------------------------------------------------
# Joint optimisation of down- and upsampling (Sec. 3.3, Alg. 2)
# --------------------------------------------------------------------------
def ccl8(mask: np.ndarray):
    """8-connected components of a boolean mask.

    Returns (labels, M): labels is int32 with 0 for background and 1..M for
    components numbered in the raster order of their first pixel.
    """
    mask = np.asarray(mask, dtype=bool)
    H, W = mask.shape
    labels = np.zeros((H, W), dtype=np.int32)
    M = 0
    for start in np.flatnonzero(mask):
        y0, x0 = divmod(int(start), W)
        if labels[y0, x0]:
            continue
        M += 1
        labels[y0, x0] = M
        queue = deque([(y0, x0)])
        while queue:
            y, x = queue.popleft()
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    ny, nx = y + dy, x + dx
                    if 0 <= ny < H and 0 <= nx < W and mask[ny, nx] and not labels[ny, nx]:
                        labels[ny, nx] = M
                        queue.append((ny, nx))
    return labels, M


@dataclass
class Decision:
    round: int
    first_pixel: int
    accepted: bool
    e0: float
    e1: float
    q_pstar: list  # [(q, p_star), ...] in ascending q


@dataclass
class JointResult:
    L: np.ndarray  # optimised LR guide (h, w, 3), float64 copies of I pixels
    a: np.ndarray
    b: np.ndarray
    alpha: np.ndarray
    err: np.ndarray
    rounds_run: int = 0
    n_large: list = field(default_factory=list)
    n_components: list = field(default_factory=list)
    n_accepted: list = field(default_factory=list)
    err_sum_initial: float = 0.0
    err_sum_final: float = 0.0
    log: list = field(default_factory=list)


def _affected_pixels(Q, h, w, H, W, s, k):
    """A = {p : Omega(p) contains some q of Q}: pixels whose cell is within r of Q."""
    r = k // 2
    cells = np.zeros((h, w), dtype=bool)
    for q in Q:
        qy, qx = divmod(int(q), w)
        cells[max(0, qy - r) : qy + r + 1, max(0, qx - r) : qx + r + 1] = True
    ys, xs = np.divmod(np.arange(H * W, dtype=np.int64), W)
    sel = cells[ys // s, xs // s]
    return np.flatnonzero(sel)


def _components_in_raster_order(large, H, W):
    """The 8-connected components of the large-error mask, each as its flat
    HR indices in ascending order, listed by their first pixel (Alg. 2
    clusters the large-error set once per iteration)."""
    labels, M = ccl8(large.reshape(H, W))
    flat = labels.ravel()
    members = np.flatnonzero(flat)
    comps = [[] for _ in range(M)]
    for p in members:
        comps[flat[p] - 1].append(int(p))
    return [np.asarray(c, dtype=np.int64) for c in comps]


@dataclass
class _JointState:
    """What Alg. 2 updates in place: I_down (flat view Lf of L) and the
    search result (a, b, alpha, E) of every HR pixel."""

    I: np.ndarray
    L: np.ndarray
    Lf: np.ndarray
    If: np.ndarray
    a: np.ndarray
    b: np.ndarray
    alpha: np.ndarray
    E: np.ndarray
    cell_of: np.ndarray  # LR cell under each HR pixel


def _component_trial(st, C, n, s, k, eps, mode, reading, decide):
    """One trial of Alg. 2 for the component C (flat HR indices, ascending).

    Q is the set of LR cells under C.  Every I_down[q] becomes the colour of
    the pixel of C in q's block with the largest current error (first such
    in HR order).  The pixels named by the reading (the affected set, whose
    windows reach Q, or C itself) are searched again; the trial stays when
    their summed error did not grow, else I_down and their search results
    are restored.  Returns the Decision."""
    H, W = st.I.shape[:2]
    h, w = st.L.shape[:2]
    Q = np.unique(st.cell_of[C])
    if reading == "affected":
        R = _affected_pixels(Q, h, w, H, W, s, k)
    elif reading == "literal":
        R = C
    else:
        raise ValueError("reading must be 'affected' or 'literal'")
    saved_L = st.Lf[Q].copy()
    saved = (st.a[R].copy(), st.b[R].copy(), st.alpha[R].copy(), st.E[R].copy())
    e0 = float(st.E[R].sum())
    q_pstar = []
    for q in Q:
        members = C[st.cell_of[C] == q]  # ascending HR index
        Em = st.E[members]
        pstar = int(members[int(np.argmax(Em))])  # first maximum
        if decide is not None:
            pstar = decide("argmax", (int(q), members, Em), pstar)
        q_pstar.append((int(q), pstar))
    for q, pstar in q_pstar:
        st.Lf[q] = st.If[pstar]
    rs = search(st.I, st.L, s, k, eps, mode, pixels=R)
    st.a[R], st.b[R], st.alpha[R], st.E[R] = rs.a, rs.b, rs.alpha, rs.err
    e1 = float(st.E[R].sum())
    keep = not (e1 > e0)
    if decide is not None:
        keep = decide("accept", (e0, e1, R.size), keep)
    if not keep:
        st.Lf[Q] = saved_L
        st.a[R], st.b[R], st.alpha[R], st.E[R] = saved
    return Decision(n, int(C[0]), keep, e0, e1, q_pstar)


def joint_downsample(
    I,
    L0,
    s,
    k=WINDOW,
    eps=EPS,
    mode="exhaustive",
    tau=TAU,
    max_iter=N_ITER,
    reading="affected",
    decide=None,
) -> JointResult:
    """Joint optimisation of down- and upsampling (Sec. 3.3, Alg. 2).

    I_down starts at ``L0`` (regular-grid downsampling by default) and
    Theta, E at the search on it.  Each of up to ``max_iter`` iterations
    takes the pixels with E > tau (none: stop), clusters them into
    8-connected components, and runs one trial per component in the order of
    their first pixels (``_component_trial``), each trial seeing the ones
    before it.  ``decide`` (optional) is called as decide(kind, payload,
    default) at each decision so a test can replay another implementation's
    near-tie decisions; it must return the decision to take.
    """
    I = np.asarray(I, dtype=np.float64)
    H, W = I.shape[:2]
    L = np.array(L0, dtype=np.float64, copy=True)
    h, w = L.shape[:2]
    r0 = search(I, L, s, k, eps, mode)
    ys, xs = np.divmod(np.arange(H * W, dtype=np.int64), W)
    st = _JointState(I=I, L=L, Lf=L.reshape(h * w, -1), If=I.reshape(H * W, -1), a=r0.a.copy(), b=r0.b.copy(),
                     alpha=r0.alpha.copy(), E=r0.err.copy(), cell_of=(ys // s) * w + (xs // s))
    res = JointResult(L=L, a=st.a, b=st.b, alpha=st.alpha, err=st.E, err_sum_initial=float(st.E.sum()))
    for n in range(1, max_iter + 1):
        large = st.E > tau
        if decide is not None:
            large = decide("membership", st.E, large)
        if not large.any():
            break
        comps = _components_in_raster_order(large, H, W)
        res.rounds_run = n
        res.n_large.append(int(large.sum()))
        res.n_components.append(len(comps))
        kept = 0
        for C in comps:
            d = _component_trial(st, C, n, s, k, eps, mode, reading, decide)
            kept += int(d.accepted)
            res.log.append(d)
        res.n_accepted.append(kept)
    res.err_sum_final = float(st.E.sum())
    return res


# --------------------------------------------------------------------------
# Gradient-driven joint downsampling (not in the paper)
# --------------------------------------------------------------------------
# An alternative to the trial replacements of Alg. 2, defined here rather
# than taken from the paper: the LR guide moves along the gradient of the
# self-upsampling error (Sec. 3.3 upsamples I_down itself and measures
# ||I_hat - I||) through Eq. 1 with Theta held fixed, and every LR pixel is
# then put back on a copy of one HR pixel of its own block, which keeps the
# one-pixel-per-LR-pixel property of Sec. 3.3.
def self_upsampling_gradient(I, L, a, b, alpha):
    """D = d/dL of sum_p ||I_hat_p - I_p||^2 with I_hat = Eq. 1 applied to L
    (Theta = (a, b, alpha) held fixed): G = 2 (I_hat - I), then the
    gradient of Eq. 1 with respect to its LR target.  Returns (D (h, w, 3),
    I_hat (H, W, 3))."""
    I = np.asarray(I, dtype=np.float64)
    L = np.asarray(L, dtype=np.float64)
    H, W = I.shape[:2]
    I_hat = apply(a, b, alpha, L).reshape(H, W, -1)
    G = 2.0 * (I_hat - I)
    _, dL = apply_backward(a, b, alpha, L, G)
    return dL.reshape(L.shape), I_hat


def snap_to_block(I, Z, s, decide=None):
    """For every LR cell q, the HR pixel of its block {p : p_down = q} whose
    colour is nearest to Z_q (squared Euclidean distance; ties to the
    smallest HR linear index).  Returns the flat HR indices (h * w,)."""
    I = np.asarray(I, dtype=np.float64)
    Z = np.asarray(Z, dtype=np.float64)
    H, W = I.shape[:2]
    h, w = Z.shape[:2]
    If = I.reshape(H * W, -1)
    out = np.empty(h * w, dtype=np.int64)
    for qy in range(h):
        ys = np.arange(qy * s, min(H, qy * s + s))
        for qx in range(w):
            xs = np.arange(qx * s, min(W, qx * s + s))
            members = (ys[:, None] * W + xs[None, :]).ravel()  # ascending HR index
            dist = ((If[members] - Z[qy, qx]) ** 2).sum(axis=1)
            p = int(members[int(np.argmin(dist))])  # first minimum
            if decide is not None:
                p = decide("snap", (qy * w + qx, members, dist), p)
            out[qy * w + qx] = p
    return out


@dataclass
class GradientJointResult:
    L: np.ndarray
    a: np.ndarray
    b: np.ndarray
    alpha: np.ndarray
    err: np.ndarray
    err_sums: list = field(default_factory=list)  # sum of E after 0, 1, ... steps
    best_step: int = 0


def joint_downsample_gradient(I, L0, s, k=WINDOW, eps=EPS, mode="exhaustive", eta=0.01, n_steps=3,
                              keep_best=True, decide=None) -> GradientJointResult:
    """Alternate the pair search with projected gradient steps on I_down.

    From L = L0 and (Theta, E) = search(I, L), each step computes
    D = self_upsampling_gradient(I, L, Theta), moves Z = L - eta D, sets
    every L_q to the HR pixel of its block nearest to Z_q (snap_to_block)
    and searches again.  Returns the L with the smallest sum of E seen (the
    first such on equality) when keep_best, else the last one, with its
    Theta and E and the sum of E after every step."""
    I = np.asarray(I, dtype=np.float64)
    H, W = I.shape[:2]
    L = np.array(L0, dtype=np.float64, copy=True)
    h, w = L.shape[:2]
    If = I.reshape(H * W, -1)
    r = search(I, L, s, k, eps, mode)
    best = (float(r.err.sum()), L.copy(), r, 0)
    sums = [best[0]]
    for t in range(1, n_steps + 1):
        D, _ = self_upsampling_gradient(I, L, r.a, r.b, r.alpha)
        Z = L - eta * D
        pick = snap_to_block(I, Z, s, decide)
        L = If[pick].reshape(h, w, -1).copy()
        r = search(I, L, s, k, eps, mode)
        e = float(r.err.sum())
        sums.append(e)
        if e < best[0]:
            best = (e, L.copy(), r, t)
    if keep_best:
        e, L, r, t_best = best
    else:
        t_best = n_steps
    return GradientJointResult(L=L, a=r.a, b=r.b, alpha=r.alpha, err=r.err, err_sums=sums, best_step=t_best)


# --------------------------------------------------------------------------
# Evaluation of given pairs (for judging another implementation's choice)
# --------------------------------------------------------------------------
def eval_pairs_exhaustive(I, L, pixels, a, b, eps=EPS):
    """Eq. 4 weight (clamped, weight on a; 1 when a == b or a zero
    denominator) and the error of the given pairs at the given pixels."""
    I = np.asarray(I, dtype=np.float64)
    L = np.asarray(L, dtype=np.float64)
    W = I.shape[1]
    ys, xs = np.divmod(np.asarray(pixels, dtype=np.int64).ravel(), W)
    Ip = I[ys, xs]
    Lf = L.reshape(-1, L.shape[2])
    La, Lb = Lf[np.asarray(a)], Lf[np.asarray(b)]
    e = La - Lb
    den = np.einsum("nc,nc->n", e, e) + eps
    g = np.einsum("nc,nc->n", Ip - Lb, e)
    with np.errstate(divide="ignore", invalid="ignore"):
        al = np.where(den > 0, np.clip(g / np.where(den > 0, den, 1.0), 0.0, 1.0), 1.0)
    al = np.where(np.asarray(a) == np.asarray(b), 1.0, al)
    rec = al[:, None] * La + (1 - al)[:, None] * Lb
    return al, np.sqrt(np.einsum("nc,nc->n", rec - Ip, rec - Ip))


def eval_pairs_fast(I, L, pixels, a, b, eps=EPS):
    """Eq. 5 weight on the anchor a (1 when b == a) and the error of (a, b)."""
    I = np.asarray(I, dtype=np.float64)
    L = np.asarray(L, dtype=np.float64)
    W = I.shape[1]
    ys, xs = np.divmod(np.asarray(pixels, dtype=np.int64).ravel(), W)
    Ip = I[ys, xs]
    Lf = L.reshape(-1, L.shape[2])
    La, Lb = Lf[np.asarray(a)], Lf[np.asarray(b)]
    da = np.linalg.norm(Ip - La, axis=1)
    db = np.linalg.norm(Ip - Lb, axis=1)
    den = da + db + eps
    with np.errstate(divide="ignore", invalid="ignore"):
        om = np.where(den > 0, db / np.where(den > 0, den, 1.0), 1.0)
    om = np.where(np.asarray(a) == np.asarray(b), 1.0, om)
    rec = om[:, None] * La + (1 - om)[:, None] * Lb
    return om, np.sqrt(np.einsum("nc,nc->n", rec - Ip, rec - Ip))


def search_fast_given_anchor(I, L, s, k, eps, pixels, anchor):
    """Second step of Algorithm 1 with the anchor a given per pixel."""
    I = np.asarray(I, dtype=np.float64)
    L = np.asarray(L, dtype=np.float64)
    H, W = I.shape[:2]
    h, w = L.shape[:2]
    ys, xs = _pixel_coords(H, W, pixels)
    Ip = I[ys, xs]
    Lf = L.reshape(-1, L.shape[2])
    cand = _candidates(ys, xs, s, h, w, k)
    anchor = np.asarray(anchor, dtype=np.int64).ravel()
    La = Lf[anchor]
    da = np.linalg.norm(Ip - La, axis=1)
    n = Ip.shape[0]
    best = np.full(n, np.inf)
    b = np.full(n, -1, dtype=np.int64)
    omega = np.full(n, np.nan)
    for v, lin in cand:
        Lb = Lf[lin]
        db = np.linalg.norm(Ip - Lb, axis=1)
        den = da + db + eps
        with np.errstate(divide="ignore", invalid="ignore"):
            om = np.where(den > 0, db / np.where(den > 0, den, 1.0), 1.0)
        om = np.where(lin == anchor, 1.0, om)
        rec = om[:, None] * La + (1.0 - om)[:, None] * Lb
        err = np.sqrt(np.einsum("nc,nc->n", rec - Ip, rec - Ip))
        upd = v & (err < best)
        best = np.where(upd, err, best)
        b = np.where(upd, lin, b)
        omega = np.where(upd, om, omega)
    return SearchResult(a=anchor, b=b, alpha=omega, err=best, pixels=np.asarray(pixels))
