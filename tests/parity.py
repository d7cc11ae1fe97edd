"""Parity protocol between the GPU path (float32) and the float64 oracle.

Per pixel (exhaustive mode):
  1. GPU pair == oracle pair: |alpha_gpu - alpha_or| <= 1e-5.
  2. otherwise the choice must be a near-tie: the oracle evaluates the GPU's
     pair (err') and requires err' - err_or <= 1e-6 (Euclidean, not
     squared); alpha is then checked against the oracle's weight for the
     GPU's pair.
Fast mode applies rule 2 first to the anchor (colour-distance gap), then to
b given the GPU's anchor; GNU mode to its anchor (b = a, weight 1).  E (when returned) must match the oracle's error
of the GPU's pair to 1e-6, and T_hat the oracle's Eq. 1 with the GPU's
pair and the oracle's weight for it to 1e-5 (float32) or one half-precision
ulp + 1e-5 (float16).
"""
from __future__ import annotations

import concurrent.futures as cf
import multiprocessing as mp
import os

import numpy as np

import oracle as O

ALPHA_TOL = 1e-5
TIE_TOL = 1e-6
T_TOL = 1e-5
E_TOL = 1e-6


def decode_codes(code, H, W, s, k, pixels):
    """Absolute LR indices (a, b) from uint16 codes (format of include/glu.h)."""
    w = -(-W // s)
    h = -(-H // s)
    code = np.asarray(code).astype(np.int64) & 0xFFFF
    K2 = k * k
    r = k // 2
    ys, xs = np.divmod(np.asarray(pixels, dtype=np.int64), W)
    cd = code.reshape(-1)[pixels]
    oa, ob = np.divmod(cd, K2)
    qy, qx = ys // s, xs // s
    a = (qy + oa // k - r) * w + (qx + oa % k - r)
    b = (qy + ob // k - r) * w + (qx + ob % k - r)
    def inside(o):
        cy, cx = qy + o // k - r, qx + o % k - r
        return (o < K2) & (cy >= 0) & (cy < h) & (cx >= 0) & (cx < w)

    valid_a = inside(oa)
    valid_b = inside(ob)
    return a, b, valid_a & valid_b


def _in_window(a, pixels, W, s, k, h, w):
    ys, xs = np.divmod(np.asarray(pixels, dtype=np.int64), W)
    qy, qx = ys // s, xs // s
    ay, ax = np.divmod(a, w)
    r = k // 2
    return (np.abs(ay - qy) <= r) & (np.abs(ax - qx) <= r) & (ay >= 0) & (ay < h) & (ax >= 0) & (ax < w)


class ParityReport(dict):
    pass


def check_search(I, L, s, k, eps, mode, code, alpha, err=None, pixels=None, T_low=None, T_hat=None,
                 out_dtype=np.float32, degenerate=True, ref=None):
    """Runs the oracle on `pixels` (default all) and checks the GPU outputs.

    I, L, T_low: host arrays of the exact values the GPU consumed.
    code, alpha, err, T_hat: host copies of the GPU outputs (full images).
    ref: the oracle's search result over `pixels` when it was computed
    already (OraclePool.search); it is updated in place.
    Returns a report dict; raises AssertionError on a violation.
    """
    I = np.asarray(I)
    H, W = I.shape[:2]
    h, w = L.shape[:2]
    if pixels is None:
        pixels = np.arange(H * W, dtype=np.int64)
    pixels = np.asarray(pixels, dtype=np.int64)
    rep = ParityReport(n=int(pixels.size), near_ties=0)
    if pixels.size == 0:
        return rep
    a_g, b_g, ok = decode_codes(code, H, W, s, k, pixels)
    assert ok.all(), "GPU codes point outside the LR image at %d pixels" % int((~ok).sum())
    assert _in_window(a_g, pixels, W, s, k, h, w).all() and _in_window(b_g, pixels, W, s, k, h, w).all()
    al_g = np.asarray(alpha, dtype=np.float64).reshape(-1)[pixels]
    if ref is not None:
        assert degenerate and ref.a.shape == pixels.shape
    elif degenerate:
        ref = O.search(I, L, s, k, eps, mode, pixels=pixels)
    else:
        assert mode == "exhaustive", "the pairs-only candidate set is an exhaustive-search option"
        ref = O.search_exhaustive(I, L, s, k, eps, pixels=pixels, degenerate=False)
    if mode == "gnu":
        # the anchor alone: a near-tie of the nearest colour, b = a, weight 1
        Lf = np.asarray(L, dtype=np.float64).reshape(-1, 3)
        ys, xs = np.divmod(pixels, W)
        Ip = np.asarray(I, dtype=np.float64)[ys, xs]
        d_g = np.linalg.norm(Ip - Lf[a_g], axis=1)
        gap = d_g - ref.err
        assert not (gap > TIE_TOL).any(), "non-tie GNU anchor, worst gap %.3g" % float(gap.max())
        assert np.array_equal(a_g, b_g) and np.all(al_g == 1.0)
        rep["near_ties"] = int((a_g != ref.a).sum())
        al_ref = np.ones_like(al_g)
        e_ref = d_g
    elif mode == "exhaustive":
        assert np.all(a_g <= b_g), "exhaustive codes must have a <= b"
        same = (a_g == ref.a) & (b_g == ref.b)
        al_ref = np.where(same, ref.alpha, 0.0)
        e_ref = ref.err.copy()
        if (~same).any():
            idx = np.flatnonzero(~same)
            al2, e2 = O.eval_pairs_exhaustive(I, L, pixels[idx], a_g[idx], b_g[idx], eps)
            gap = e2 - ref.err[idx]
            bad = gap > TIE_TOL
            assert not bad.any(), (
                "non-tie pair mismatch at %d pixels, worst gap %.3g (pixel %d)"
                % (int(bad.sum()), float(gap.max()), int(pixels[idx][np.argmax(gap)]))
            )
            al_ref[idx] = al2
            e_ref[idx] = e2
            rep["near_ties"] = int(idx.size)
    else:
        # anchor first: the GPU anchor must be (nearly) as close as the oracle's
        Lf = np.asarray(L, dtype=np.float64).reshape(-1, 3)
        ys, xs = np.divmod(pixels, W)
        Ip = np.asarray(I, dtype=np.float64)[ys, xs]
        da_g = np.linalg.norm(Ip - Lf[a_g], axis=1)
        da_o = np.linalg.norm(Ip - Lf[ref.a], axis=1)
        gap_a = da_g - da_o
        assert not (gap_a > TIE_TOL).any(), "non-tie anchor mismatch, worst gap %.3g" % float(gap_a.max())
        diff_a = a_g != ref.a
        if diff_a.any():
            idx = np.flatnonzero(diff_a)
            r2 = O.search_fast_given_anchor(I, L, s, k, eps, pixels[idx], a_g[idx])
            for f in ("b", "alpha", "err"):
                getattr(ref, f)[idx] = getattr(r2, f)[...]
            ref.a[idx] = a_g[idx]
        same = b_g == ref.b
        al_ref = np.where(same, ref.alpha, 0.0)
        e_ref = ref.err.copy()
        if (~same).any():
            idx = np.flatnonzero(~same)
            al2, e2 = O.eval_pairs_fast(I, L, pixels[idx], a_g[idx], b_g[idx], eps)
            gap = e2 - ref.err[idx]
            bad = gap > TIE_TOL
            assert not bad.any(), (
                "non-tie partner mismatch at %d pixels, worst gap %.3g" % (int(bad.sum()), float(gap.max()))
            )
            al_ref[idx] = al2
            e_ref[idx] = e2
        rep["near_ties"] = int((~same).sum() + diff_a.sum())
    da = np.abs(al_g - al_ref)
    assert da.max() <= ALPHA_TOL, "alpha error %.3g > %.1g at pixel %d" % (
        float(da.max()), ALPHA_TOL, int(pixels[np.argmax(da)]))
    assert np.all((al_g >= 0) & (al_g <= 1))
    rep["alpha_max_err"] = float(da.max())
    if err is not None:
        e_g = np.asarray(err, dtype=np.float64).reshape(-1)[pixels]
        de = np.abs(e_g - e_ref)
        assert de.max() <= E_TOL, "E error %.3g at pixel %d" % (float(de.max()), int(pixels[np.argmax(de)]))
        rep["err_max_err"] = float(de.max())
    if T_hat is not None:
        Cn = T_low.shape[2]
        ref_T = O.apply(a_g, b_g, al_ref, T_low)
        got = np.asarray(T_hat, dtype=np.float64).reshape(-1, Cn)[pixels]
        dT = np.abs(got - ref_T)
        if out_dtype == np.float16:
            tol = np.abs(np.spacing(ref_T.astype(np.float16))).astype(np.float64) + T_TOL
            assert np.all(dT <= tol), "T_hat fp16 error %.3g" % float(dT.max())
        else:
            assert dT.max() <= T_TOL, "T_hat error %.3g at pixel %d" % (
                float(dT.max()), int(pixels[np.argmax(dT.max(axis=1))]))
        rep["T_max_err"] = float(dT.max())
    return rep


# ---------------------------------------------------------------------------
# The oracle's search over many pixels, split across host processes.
# ---------------------------------------------------------------------------

def _pool_job(job):
    """Worker side: the oracle's search of one chunk of pixels, all of them
    in rows y0 .. y0 + len(rows) - 1 of an H x W image.  The search reads the
    guide only at the searched pixels (and the LR guide in their windows), so
    the worker places the rows into an otherwise empty full-size image (its
    untouched pages are never allocated)."""
    H, W, y0, rows, L, s, k, eps, mode, pix = job
    I = np.zeros((H, W, rows.shape[2]), dtype=np.float64)
    I[y0:y0 + rows.shape[0]] = rows
    r = O.search(I, L, s, k, eps, mode, pixels=pix)
    return r.a, r.b, r.alpha, r.err


def pool_workers():
    """Host cores this process may use, at most 16."""
    return max(1, min(16, len(os.sched_getaffinity(0))))


class OraclePool:
    """A pool of spawned processes that run the oracle's search (they import
    numpy and the oracle only, and never touch the GPU).  ``search`` returns
    what one ``O.search`` call over the same pixels returns."""

    def __init__(self, workers=None):
        self.workers = workers or pool_workers()
        self._ex = cf.ProcessPoolExecutor(self.workers, mp_context=mp.get_context("spawn"))

    def close(self):
        self._ex.shutdown(wait=True, cancel_futures=True)

    def search(self, I, L, s, k, eps, mode, pixels=None, chunk=1 << 16):
        I = np.asarray(I)
        H, W = I.shape[:2]
        if pixels is None:
            pixels = np.arange(H * W, dtype=np.int64)
        pixels = np.asarray(pixels, dtype=np.int64)
        n_chunks = max(1, min(-(-pixels.size // chunk), 64 * self.workers))
        jobs = []
        for pix in np.array_split(pixels, n_chunks):
            if pix.size == 0:
                continue
            ys = pix // W
            y0, y1 = int(ys.min()), int(ys.max()) + 1
            jobs.append((H, W, y0, np.asarray(I[y0:y1]), np.asarray(L), s, k, eps, mode, pix))
        try:
            parts = list(self._ex.map(_pool_job, jobs))
        except cf.process.BrokenProcessPool:
            self._ex.shutdown(wait=False, cancel_futures=True)
            raise
        if not parts:
            e = np.zeros(0)
            return O.SearchResult(a=e.astype(np.int64), b=e.astype(np.int64), alpha=e, err=e, pixels=pixels)
        cat = lambda i: np.concatenate([p[i] for p in parts])
        return O.SearchResult(a=cat(0), b=cat(1), alpha=cat(2), err=cat(3), pixels=pixels)
