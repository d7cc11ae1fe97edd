"""Python binding of libglu: torch tensors in, torch tensors out.

Argument marshalling only: every step runs in the HIP kernels behind the C
ABI of include/glu.h.  Tensors must live on the GPU; images are (H, W, C)
with the channel axis innermost (rows may be padded).  Theta is returned as a
``Theta`` pair of (H, W) tensors: ``code`` (int16 holding the uint16 codes)
and ``alpha`` (float32).  All calls run on torch's current stream.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import torch

from . import _lib as L

EPS = 1e-3  # Eq. 4 regulariser (Sec. 3.1)
TAU = 30.0 / 255.0  # error threshold of Algorithm 2 (Sec. 5.2)
N_ITER = 3  # iterations of Algorithm 2 (Sec. 5.2)

_MODES = {"exhaustive": L.GLU_SEARCH_EXHAUSTIVE, "fast": L.GLU_SEARCH_FAST, "gnu": L.GLU_SEARCH_GNU}


@dataclass
class Theta:
    code: torch.Tensor  # (H, W) int16 view of the uint16 codes
    alpha: torch.Tensor  # (H, W) float32

    @property
    def shape(self):
        return tuple(self.code.shape)


# torch's raw current-stream query (no Stream object per call); the public
# form is the fallback
_RAW_STREAM = getattr(torch._C, "_cuda_getCurrentRawStream", None)
_GET_DEVICE = getattr(torch._C, "_cuda_getDevice", None)


def _stream():
    if _RAW_STREAM is not None and _GET_DEVICE is not None:
        return C.c_void_p(_RAW_STREAM(_GET_DEVICE()))
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


_DTYPES = {torch.float32: L.GLU_F32, torch.float16: L.GLU_F16}


def _dtype_code(t: torch.Tensor) -> int:
    code = _DTYPES.get(t.dtype)
    if code is None:
        raise TypeError("images must be float32 or float16, got %s" % t.dtype)
    return code


def _img(t: torch.Tensor, name: str) -> L.glu_image:
    if not isinstance(t, torch.Tensor) or t.dim() != 3:
        raise ValueError("%s must be an (H, W, C) tensor" % name)
    if not t.is_cuda:
        raise ValueError("%s must be a GPU tensor" % name)
    H, W, Cn = t.shape
    st = t.stride()
    if H * W > 0 and not (st[2] == 1 and (W <= 1 or st[1] == Cn)):
        raise ValueError("%s rows must be dense (channels innermost, pixels adjacent)" % name)
    stride = st[0] if H > 1 else W * Cn
    return L.glu_image(t.data_ptr() if H * W * Cn else None, H, W, Cn, max(stride, W * Cn), _dtype_code(t))


def _theta(th: Theta) -> L.glu_theta:
    code, alpha = th.code, th.alpha
    if code.dtype != torch.int16 or alpha.dtype != torch.float32:
        raise TypeError("theta must be (int16 code, float32 alpha)")
    if code.shape != alpha.shape or code.dim() != 2:
        raise ValueError("theta code and alpha must both be (H, W)")
    H, W = code.shape
    st = code.stride()
    if st != alpha.stride() or (H * W and st[1] != 1):
        raise ValueError("theta code and alpha must share a row-major layout")
    stride = st[0] if H > 1 else W
    n = H * W
    return L.glu_theta(code.data_ptr() if n else None, alpha.data_ptr() if n else None, H, W, max(stride, W))


def _per_pixel(buf, th_desc, H: int, W: int, device, name: str):
    """A float32 (H, W) per-pixel output (E or grad_alpha) laid out with
    Theta's row stride, as the C ABI writes it: allocated that way when
    ``buf`` is None, else checked (a buffer with another row stride would be
    written out of bounds or in the wrong places)."""
    stride = th_desc.row_stride if th_desc is not None else W
    if buf is None:
        if H * W == 0:
            return torch.empty((H, W), dtype=torch.float32, device=device)
        return torch.empty((H, stride), dtype=torch.float32, device=device)[:, :W]
    if not isinstance(buf, torch.Tensor) or buf.dtype != torch.float32 or tuple(buf.shape) != (H, W):
        raise ValueError("%s must be a float32 (%d, %d) tensor" % (name, H, W))
    if not buf.is_cuda:
        raise ValueError("%s must be a GPU tensor" % name)
    if H * W and ((W > 1 and buf.stride(1) != 1) or (H > 1 and buf.stride(0) != stride)):
        raise ValueError("%s must have Theta's row stride (%d elements)" % (name, stride))
    return buf


_PARAMS: dict = {}


def _params(s: int, k: int, eps: float, mode: str = "exhaustive", degenerate: bool = True) -> L.glu_params:
    """The glu_params of one call.  The struct is read only during the call,
    so one instance per distinct argument set is kept and passed again."""
    key = (s, k, eps, mode, degenerate)
    p = _PARAMS.get(key)
    if p is None:
        if mode not in _MODES:
            raise ValueError("mode must be 'exhaustive', 'fast' or 'gnu'")
        flags = 0 if degenerate else L.GLU_FLAG_NO_DEGENERATE
        p = L.glu_params(int(s), int(k), float(eps), _MODES[mode], flags)
        if len(_PARAMS) < 256:
            _PARAMS[key] = p
    return p


def lr_shape(H: int, W: int, s: int):
    return (-(-H // s), -(-W // s))


def empty_theta(H: int, W: int, device="cuda") -> Theta:
    return Theta(
        torch.empty((H, W), dtype=torch.int16, device=device), torch.empty((H, W), dtype=torch.float32, device=device)
    )


def downsample(I: torch.Tensor, s: int, mode: str = "point", out: torch.Tensor | None = None) -> torch.Tensor:
    """Regular-grid (point) or box downsampling of I to ceil(H/s) x ceil(W/s)
    (into ``out`` when given)."""
    h, w = lr_shape(I.shape[0], I.shape[1], s)
    if out is None:
        out = torch.empty((h, w, I.shape[2]), dtype=I.dtype, device=I.device)
    m = {"point": L.GLU_DOWN_POINT, "box": L.GLU_DOWN_BOX}[mode]
    lib = L.load()
    L.check(lib.glu_downsample(C.byref(_img(I, "I")), C.byref(_img(out, "I_low")), int(s), m, _stream()))
    return out


def search(I, I_low, s, k=3, eps=EPS, mode="exhaustive", return_err=False, theta: Theta | None = None, err=None,
           degenerate=True):
    """Per-pixel (a, b, alpha) search; returns Theta (and E when return_err).
    degenerate=False (exhaustive only) keeps the pairs i < j alone as
    candidates (GLU_FLAG_NO_DEGENERATE)."""
    H, W = I.shape[:2]
    theta = theta if theta is not None else empty_theta(H, W, I.device)
    thd = _theta(theta)
    if return_err or err is not None:
        err = _per_pixel(err, thd, H, W, I.device, "err")
    p = _params(s, k, eps, mode, degenerate)
    lib = L.load()
    L.check(
        lib.glu_search(
            C.byref(_img(I, "I")),
            C.byref(_img(I_low, "I_low")),
            C.byref(p),
            C.byref(thd),
            C.c_void_p(err.data_ptr() if err is not None and err.numel() else None),
            _stream(),
        )
    )
    return (theta, err) if return_err else theta


def _batch_view(t: torch.Tensor, name: str, dims: int):
    """(first image, batch stride in elements) of a (B, ...) tensor."""
    if t.dim() != dims + 1:
        raise ValueError("%s must have a leading batch dimension" % name)
    return t[0], (t.stride(0) if t.shape[0] > 1 else 0)


def _theta_batch(th: Theta):
    if th.code.dim() != 3 or th.alpha.shape != th.code.shape or th.code.stride() != th.alpha.stride():
        raise ValueError("batched theta code and alpha must both be (B, H, W) with one layout")
    return Theta(th.code[0], th.alpha[0]), (th.code.stride(0) if th.code.shape[0] > 1 else 0)


def apply(theta: Theta, T_low: torch.Tensor, s: int, k: int = 3, out: torch.Tensor | None = None):
    """Eq. 1 with a given Theta.  T_low (h, w, C) with Theta (H, W), or a batch:
    T_low (B, h, w, C) with Theta (B, H, W), in one launch."""
    if T_low.dim() == 4:
        return _apply_batched(theta, T_low, s, k, out)
    H, W = theta.shape
    if out is None:
        out = torch.empty((H, W, T_low.shape[2]), dtype=T_low.dtype, device=T_low.device)
    p = _params(s, k, EPS)
    lib = L.load()
    L.check(
        lib.glu_apply(
            C.byref(_theta(theta)), C.byref(_img(T_low, "T_low")), C.byref(p), C.byref(_img(out, "T_hat")), _stream()
        )
    )
    return out


def _apply_batched(theta: Theta, T_low, s, k, out):
    B = T_low.shape[0]
    H, W = theta.code.shape[1:]
    if theta.code.shape[0] != B:
        raise ValueError("theta and T_low batch sizes differ")
    if out is None:
        out = torch.empty((B, H, W, T_low.shape[3]), dtype=T_low.dtype, device=T_low.device)
    if B == 0:
        return out
    th0, sth = _theta_batch(theta)
    T0, sT = _batch_view(T_low, "T_low", 3)
    o0, so = _batch_view(out, "out", 3)
    bs = L.glu_batch_strides(sth, sT, so, 0, 0)
    p = _params(s, k, EPS)
    L.check(
        L.load().glu_apply_batched(
            B, C.byref(bs), C.byref(_theta(th0)), C.byref(_img(T0, "T_low")), C.byref(p), C.byref(_img(o0, "T_hat")),
            _stream(),
        )
    )
    return out


def search_apply(
    I, I_low, T_low, s, k=3, eps=EPS, mode="exhaustive", store_theta=True, return_err=False, theta=None, out=None,
    err=None, degenerate=True,
):
    """Fused search + apply; returns (T_hat, Theta or None[, E])."""
    H, W = I.shape[:2]
    if store_theta and theta is None:
        theta = empty_theta(H, W, I.device)
    if out is None:
        out = torch.empty((H, W, T_low.shape[2]), dtype=T_low.dtype, device=I.device)
    thd = _theta(theta) if theta is not None else None
    if return_err or err is not None:
        err = _per_pixel(err, thd, H, W, I.device, "err")
    p = _params(s, k, eps, mode, degenerate)
    lib = L.load()
    th = C.byref(thd) if thd is not None else None
    L.check(
        lib.glu_search_apply(
            C.byref(_img(I, "I")),
            C.byref(_img(I_low, "I_low")),
            C.byref(_img(T_low, "T_low")),
            C.byref(p),
            th,
            C.c_void_p(err.data_ptr() if err is not None and err.numel() else None),
            C.byref(_img(out, "T_hat")),
            _stream(),
        )
    )
    return (out, theta, err) if return_err else (out, theta)


def theta_expand(theta: Theta, s: int, k: int = 3):
    """Absolute LR linear indices (a, b), int64 (H, W): the paper's 3 x H x W form with alpha."""
    H, W = theta.shape
    a = torch.empty((H, W), dtype=torch.int64, device=theta.code.device)
    b = torch.empty((H, W), dtype=torch.int64, device=theta.code.device)
    p = _params(s, k, EPS)
    lib = L.load()
    L.check(
        lib.glu_theta_expand(
            C.byref(_theta(theta)), C.byref(p), C.c_void_p(a.data_ptr() if a.numel() else None),
            C.c_void_p(b.data_ptr() if b.numel() else None), _stream()
        )
    )
    return a, b


def apply_backward_workspace(H: int, W: int, channels: int, s: int, k: int = 3) -> int:
    lib = L.load()
    p = _params(s, k, EPS)
    return int(lib.glu_apply_backward_workspace(int(H), int(W), int(channels), C.byref(p)))


def apply_backward(theta: Theta, T_low, grad_T_hat, s, k=3, need_T_low=True, need_alpha=True, workspace=None,
                   out_T_low=None, out_alpha=None):
    """Gradients of Eq. 1 (indices fixed): returns (grad_T_low or None, grad_alpha or None).

    Batched when T_low is (B, h, w, C) (Theta (B, H, W), grad_T_hat
    (B, H, W, C)): one launch per pass for the whole batch."""
    if T_low.dim() == 4:
        return _apply_backward_batched(theta, T_low, grad_T_hat, s, k, need_T_low, need_alpha, workspace, out_T_low,
                                       out_alpha)
    H, W = theta.shape
    Cn = T_low.shape[2]
    thd = _theta(theta)
    gT = None
    if need_T_low:
        gT = out_T_low if out_T_low is not None else torch.empty(
            T_low.shape, dtype=torch.float32, device=T_low.device)
    ga = None
    if need_alpha:
        ga = _per_pixel(out_alpha, thd, H, W, T_low.device, "grad_alpha")
    p = _params(s, k, EPS)
    lib = L.load()
    ws_bytes = 0
    if need_T_low:
        ws_bytes = int(lib.glu_apply_backward_workspace(H, W, Cn, C.byref(p)))
        if workspace is None or workspace.numel() * workspace.element_size() < ws_bytes:
            workspace = torch.empty(max(1, ws_bytes // 4), dtype=torch.float32, device=T_low.device)
    L.check(
        lib.glu_apply_backward(
            C.byref(thd),
            C.byref(_img(T_low, "T_low")),
            C.byref(p),
            C.byref(_img(grad_T_hat, "grad_T_hat")),
            C.byref(_img(gT, "grad_T_low")) if gT is not None else None,
            C.c_void_p(ga.data_ptr() if ga is not None and ga.numel() else None),
            C.c_void_p(workspace.data_ptr() if workspace is not None else None),
            ws_bytes,
            _stream(),
        )
    )
    return gT, ga


def apply_backward_static(theta: Theta, T_low, grad_T_hat, s, k=3, need_T_low=True, need_alpha=True, out_T_low=None,
                          out_alpha=None):
    """apply_backward through glu_apply_backward_static: no workspace and no
    allocation in the library (the outputs are allocated here when not given);
    calls on one GPU share the library's array and must not overlap."""
    H, W = theta.shape
    thd = _theta(theta)
    gT = None
    if need_T_low:
        gT = out_T_low if out_T_low is not None else torch.empty(
            T_low.shape, dtype=torch.float32, device=T_low.device)
    ga = None
    if need_alpha:
        ga = _per_pixel(out_alpha, thd, H, W, T_low.device, "grad_alpha")
    p = _params(s, k, EPS)
    L.check(
        L.load().glu_apply_backward_static(
            C.byref(thd),
            C.byref(_img(T_low, "T_low")),
            C.byref(p),
            C.byref(_img(grad_T_hat, "grad_T_hat")),
            C.byref(_img(gT, "grad_T_low")) if gT is not None else None,
            C.c_void_p(ga.data_ptr() if ga is not None and ga.numel() else None),
            _stream(),
        )
    )
    return gT, ga


def apply_backward_batched_workspace(B: int, H: int, W: int, channels: int, s: int, k: int = 3) -> int:
    lib = L.load()
    p = _params(s, k, EPS)
    return int(lib.glu_apply_backward_batched_workspace(int(B), int(H), int(W), int(channels), C.byref(p)))


def _apply_backward_batched(theta, T_low, grad_T_hat, s, k, need_T_low, need_alpha, workspace, out_T_low, out_alpha):
    B = T_low.shape[0]
    H, W = theta.code.shape[1:]
    Cn = T_low.shape[3]
    if theta.code.shape[0] != B or grad_T_hat.shape[0] != B:
        raise ValueError("theta, T_low and grad_T_hat batch sizes differ")
    gT = None
    if need_T_low:
        gT = out_T_low if out_T_low is not None else torch.empty(T_low.shape, dtype=torch.float32,
                                                                 device=T_low.device)
    ga = None
    if need_alpha:
        ga = out_alpha if out_alpha is not None else torch.empty((B, H, W), dtype=torch.float32, device=T_low.device)
    if B == 0:
        return gT, ga
    th0, sth = _theta_batch(theta)
    T0, sT = _batch_view(T_low, "T_low", 3)
    G0, sG = _batch_view(grad_T_hat, "grad_T_hat", 3)
    sgT, sga = 0, 0
    if gT is not None:
        gT0, sgT = _batch_view(gT, "grad_T_low", 3)
    if ga is not None:
        if ga.dim() != 3 or ga.shape[1:] != (H, W) or (H > 1 and ga.stride(1) != th0.code.stride(0)):
            raise ValueError("grad_alpha must be (B, H, W) with Theta's row stride")
        sga = ga.stride(0) if B > 1 else 0
    bs = L.glu_batch_strides(sth, sT, sG, sgT, sga)
    p = _params(s, k, EPS)
    lib = L.load()
    ws_bytes = 0
    if need_T_low:
        ws_bytes = int(lib.glu_apply_backward_batched_workspace(B, H, W, Cn, C.byref(p)))
        if workspace is None or workspace.numel() * workspace.element_size() < ws_bytes:
            workspace = torch.empty(max(1, ws_bytes // 4), dtype=torch.float32, device=T_low.device)
    L.check(
        lib.glu_apply_backward_batched(
            B,
            C.byref(bs),
            C.byref(_theta(th0)),
            C.byref(_img(T0, "T_low")),
            C.byref(p),
            C.byref(_img(G0, "grad_T_hat")),
            C.byref(_img(gT0, "grad_T_low")) if gT is not None else None,
            C.c_void_p(ga.data_ptr() if ga is not None and ga.numel() else None),
            C.c_void_p(workspace.data_ptr() if workspace is not None else None),
            ws_bytes,
            _stream(),
        )
    )
    return gT, ga


def joint_downsample_workspace(H: int, W: int, s: int, k: int = 3) -> int:
    lib = L.load()
    p = _params(s, k, EPS)
    return int(lib.glu_joint_downsample_workspace(int(H), int(W), C.byref(p)))


def joint_downsample(I, I_low0, s, k=3, eps=EPS, mode="exhaustive", tau=TAU, max_iter=N_ITER, log_capacity=None,
                     q_capacity=None, workspace=None):
    """Algorithm 2 (joint down/upsampling).  Returns (I_low, Theta, E, stats, log).

    I_low0 is not modified (a copy is optimised).  stats is a dict of the
    per-round counts; log a list of per-trial dicts in the sequential order
    (empty, and not recorded, when log_capacity is 0).
    """
    H, W = I.shape[:2]
    I_low = I_low0.clone()
    theta = empty_theta(H, W, I.device)
    err = torch.empty((H, W), dtype=torch.float32, device=I.device)
    p = _params(s, k, eps, mode)
    lib = L.load()
    ws_bytes = int(lib.glu_joint_downsample_workspace(H, W, C.byref(p)))
    if workspace is None or workspace.numel() * workspace.element_size() < ws_bytes:
        workspace = torch.empty(max(1, ws_bytes), dtype=torch.uint8, device=I.device)
    st = L.glu_jd_stats()
    cap = int(log_capacity if log_capacity is not None else max(1024, H * W // 16))
    qcap = int(q_capacity if q_capacity is not None else 4 * cap)
    cap, qcap = max(cap, 0), max(qcap, 0)
    arrs = dict(
        round=(C.c_int32 * cap)(), first_pixel=(C.c_int32 * cap)(), accepted=(C.c_uint8 * cap)(),
        e0=(C.c_double * cap)(), e1=(C.c_double * cap)(), n_q=(C.c_int32 * cap)(),
        q_and_pstar=(C.c_int64 * (2 * qcap))(),
    )
    lg = L.glu_jd_log(cap, 0, arrs["round"], arrs["first_pixel"], arrs["accepted"], arrs["e0"], arrs["e1"],
                      arrs["n_q"], qcap, arrs["q_and_pstar"], 0)
    L.check(
        lib.glu_joint_downsample(
            C.byref(_img(I, "I")),
            C.byref(_img(I_low, "I_low")),
            C.byref(p),
            float(tau),
            int(max_iter),
            C.byref(_theta(theta)),
            C.c_void_p(err.data_ptr() if err.numel() else None),
            C.c_void_p(workspace.data_ptr()),
            ws_bytes,
            C.byref(st),
            C.byref(lg) if cap > 0 else None,
            _stream(),
        )
    )
    n = st.rounds_run
    stats = dict(
        rounds_run=n,
        n_large=list(st.n_large[:n]),
        n_components=list(st.n_components[:n]),
        n_accepted=list(st.n_accepted[:n]),
        n_waves=list(st.n_waves[:n]),
        err_sum_initial=st.err_sum_initial,
        err_sum_final=st.err_sum_final,
    )
    log = []
    qo = 0
    for i in range(lg.count):
        nq = arrs["n_q"][i]
        pairs = [(int(arrs["q_and_pstar"][2 * (qo + j)]), int(arrs["q_and_pstar"][2 * (qo + j) + 1])) for j in range(nq)]
        qo += nq
        log.append(dict(round=arrs["round"][i], first_pixel=arrs["first_pixel"][i], accepted=bool(arrs["accepted"][i]),
                        e0=arrs["e0"][i], e1=arrs["e1"][i], q_pstar=pairs))
    if lg.truncated:
        stats["log_truncated"] = True
    return I_low, theta, err, stats, log


def joint_downsample_grad(I, I_low0, s, k=3, eps=EPS, mode="exhaustive", eta=0.01, n_steps=3, keep_best=True,
                          workspace=None):
    """Gradient-driven joint downsampling (glu_joint_downsample_grad).

    Returns (I_low, Theta, E, err_sums, best_step); I_low0 is not modified."""
    H, W = I.shape[:2]
    I_low = I_low0.clone()
    theta = empty_theta(H, W, I.device)
    err = torch.empty((H, W), dtype=torch.float32, device=I.device)
    p = _params(s, k, eps, mode)
    lib = L.load()
    ws_bytes = int(lib.glu_joint_downsample_grad_workspace(H, W, C.byref(p)))
    if workspace is None or workspace.numel() * workspace.element_size() < ws_bytes:
        workspace = torch.empty(max(256, ws_bytes), dtype=torch.uint8, device=I.device)
    sums = (C.c_double * (int(n_steps) + 1))()
    best = C.c_int32(0)
    L.check(
        lib.glu_joint_downsample_grad(
            C.byref(_img(I, "I")), C.byref(_img(I_low, "I_low")), C.byref(p), float(eta), int(n_steps),
            1 if keep_best else 0, C.byref(_theta(theta)), C.c_void_p(err.data_ptr() if err.numel() else None),
            C.c_void_p(workspace.data_ptr()), ws_bytes, sums, C.byref(best), _stream(),
        )
    )
    return I_low, theta, err, list(sums), int(best.value)


def _batch_item(it) -> L.glu_batch_item:
    th = it.get("theta")
    if th is not None:
        thd = _theta(th)
    else:
        H, W = it["I"].shape[:2]
        thd = L.glu_theta(None, None, H, W, W)
    return L.glu_batch_item(
        _img(it["I"], "I"), _img(it["I_low"], "I_low"), _img(it["T_low"], "T_low"), _img(it["T_hat"], "T_hat"), thd,
        int(it["s"]), int(it["k"]),
    )


class BatchPlan:
    """Fused search + apply over many images: one launch per kernel variant
    present (window class, pixels per strip, storage type, LDS table), one
    workgroup per tile; a batch of one variant is a single launch.

    items: list of dicts with I, I_low, T_low, T_hat (tensors), s, k and an
    optional Theta.  The tensors must stay alive while the plan is used.
    """

    def __init__(self, items, eps=EPS, mode="exhaustive", degenerate=True):
        self.items = list(items)
        arr = (L.glu_batch_item * max(1, len(self.items)))(*[_batch_item(it) for it in self.items])
        p = _params(1, 3, eps, mode, degenerate)
        lib = L.load()
        h = C.c_void_p()
        L.check(lib.glu_batch_plan_create(arr, len(self.items), C.byref(p), C.byref(h)))
        self._h = h

    def launch(self):
        L.check(L.load().glu_batch_plan_launch(self._h, _stream()))

    def info(self):
        nt, ng = C.c_int64(), C.c_int32()
        L.check(L.load().glu_batch_plan_info(self._h, C.byref(nt), C.byref(ng)))
        return int(nt.value), int(ng.value)

    def capture_graph(self):
        """Captures one launch into a torch.cuda.CUDAGraph (a hipGraph on ROCm); replay() reruns it."""
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            self.launch()  # warm-up outside capture
        torch.cuda.current_stream().wait_stream(s)
        with torch.cuda.graph(g):
            self.launch()
        return g

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            L.load().glu_batch_plan_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune(item, eps=EPS, mode="exhaustive") -> int:
    """Times the tile variants for the item's (mode, k, s, dtype) and records the fastest."""
    lib = L.load()
    arr = (L.glu_batch_item * 1)(_batch_item(item))
    p = _params(1, 3, eps, mode)
    v = C.c_int32()
    L.check(lib.glu_autotune(arr, C.byref(p), C.byref(v), _stream()))
    return int(v.value)


def autotune_save(path: str):
    L.check(L.load().glu_autotune_save(path.encode()))


def autotune_load(path: str):
    L.check(L.load().glu_autotune_load(path.encode()))


class GluApply(torch.autograd.Function):
    """Eq. 1 as an autograd function of (alpha, T_low); the codes are constant.

    forward(alpha, T_low, code, s, k) -> T_hat.  The backward is the
    hand-written deterministic gather of glu_apply_backward.  With a batch
    dimension (alpha and code (B, H, W), T_low (B, h, w, C)) forward and
    backward each run the whole batch in one launch per pass.
    """

    @staticmethod
    def forward(ctx, alpha, T_low, code, s, k=3):
        th = Theta(code, alpha.contiguous())
        out = apply(th, T_low.contiguous(), s, k)
        ctx.save_for_backward(code, th.alpha, T_low)
        ctx.s, ctx.k = s, k
        return out

    @staticmethod
    def backward(ctx, grad_out):
        code, alpha, T_low = ctx.saved_tensors
        g = grad_out.contiguous().float()
        gT, ga = apply_backward(
            Theta(code, alpha), T_low, g, ctx.s, ctx.k, ctx.needs_input_grad[1], ctx.needs_input_grad[0]
        )
        return ga, gT, None, None, None


def glu_apply_autograd(alpha, T_low, code, s, k=3):
    return GluApply.apply(alpha, T_low, code, s, k)
