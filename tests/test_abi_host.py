"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/glu.h declares, and rejects invalid arguments before
enqueuing anything."""
import ctypes as C
import os
import re

import pytest

from paper_2307_09582_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    hdr = open(os.path.join(ROOT, "include", "glu.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    names = re.findall(r"\b(glu_[a-z0-9_]+)\s*\(", hdr)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    lib = L.load()
    names = _declared_functions()
    assert len(names) >= 18
    for n in names:
        assert hasattr(lib, n), "missing export " + n
    assert set(names) == set(L._SIGS), "binding signatures out of sync with glu.h"


def test_status_strings():
    lib = L.load()
    for code, name in L.STATUS_NAMES.items():
        assert lib.glu_status_string(code).decode() == name
    assert lib.glu_version().decode().startswith("glu-mi355x")


def _img(ptr=0x1000, H=8, W=8, Cn=3, stride=None, dt=L.GLU_F32):
    return L.glu_image(ptr, H, W, Cn, stride if stride is not None else W * Cn, dt)


def _params(s=4, k=3, eps=1e-3, mode=0, flags=0):
    return L.glu_params(s, k, eps, mode, flags)


def _theta(H=8, W=8, code=0x2000, alpha=0x3000):
    return L.glu_theta(code, alpha, H, W, W)


def _search(I, Il, p, th):
    lib = L.load()
    return lib.glu_search(
        C.byref(I) if I is not None else None,
        C.byref(Il) if Il is not None else None,
        C.byref(p) if p is not None else None,
        C.byref(th) if th is not None else None,
        None,
        None,
    )


@pytest.mark.parametrize(
    "kw,expect",
    [
        (dict(p=None), 1),
        (dict(I=None), 1),
        (dict(p=_params(s=0)), 4),
        (dict(p=_params(k=4)), 4),
        (dict(p=_params(k=17)), 4),
        (dict(p=_params(eps=-1.0)), 4),
        (dict(p=_params(eps=float("nan"))), 4),
        (dict(p=_params(mode=7)), 4),
        (dict(p=_params(flags=2)), 4),
        (dict(p=_params(mode=1, flags=1)), 4),
        (dict(p=_params(mode=2, flags=1)), 4),
        (dict(I=_img(Cn=4)), 2),
        (dict(Il=_img(H=3, W=2)), 2),
        (dict(Il=_img(H=2, W=2, dt=L.GLU_F16)), 3),
        (dict(I=_img(dt=9)), 3),
        (dict(I=_img(ptr=0x1001)), 5),
        (dict(I=_img(stride=5)), 2),
        (dict(th=_theta(H=7)), 2),
        (dict(th=_theta(code=0)), 1),
        (dict(I=_img(ptr=0)), 1),
    ],
)
def test_search_validation(kw, expect):
    args = dict(I=_img(), Il=_img(H=2, W=2), p=_params(), th=_theta())
    args.update(kw)
    st = _search(args["I"], args["Il"], args["p"], args["th"])
    assert st == expect, L.load().glu_last_error()
    assert L.load().glu_last_error().decode().startswith(L.STATUS_NAMES[expect])


def test_apply_validation():
    lib = L.load()
    th = _theta()
    p = _params()
    # T_low with the wrong LR size
    st = lib.glu_apply(C.byref(th), C.byref(_img(H=3, W=2, Cn=1)), C.byref(p), C.byref(_img(Cn=1)), None)
    assert st == 2
    # channel counts differ
    st = lib.glu_apply(C.byref(th), C.byref(_img(H=2, W=2, Cn=1)), C.byref(p), C.byref(_img(Cn=2)), None)
    assert st == 2
    # more than 4 channels
    st = lib.glu_apply(C.byref(th), C.byref(_img(H=2, W=2, Cn=5)), C.byref(p), C.byref(_img(Cn=5)), None)
    assert st == 2


def test_downsample_and_expand_validation():
    lib = L.load()
    assert lib.glu_downsample(C.byref(_img()), C.byref(_img(H=2, W=2)), 0, 0, None) == 4
    assert lib.glu_downsample(C.byref(_img()), C.byref(_img(H=2, W=2)), 4, 5, None) == 4
    assert lib.glu_downsample(C.byref(_img()), C.byref(_img(H=3, W=2)), 4, 0, None) == 2
    th = _theta()
    assert lib.glu_theta_expand(C.byref(th), C.byref(_params()), None, None, None) == 1
    assert lib.glu_theta_expand(C.byref(th), C.byref(_params()), 0x1004, 0x2000, None) == 5


def test_empty_images_return_ok_without_launch():
    # zero pixels: valid arguments, nothing to do, no HIP call is made
    st = _search(_img(ptr=0, H=0, W=5), _img(ptr=0, H=0, W=2), _params(), _theta(H=0, W=5, code=0, alpha=0))
    assert st == 0


def test_batched_validation():
    lib = L.load()
    th = _theta()
    p = _params()
    Tl = _img(H=2, W=2, Cn=1)
    Th = _img(Cn=1)
    bs = L.glu_batch_strides(64, 4, 64, 0, 0)
    # batch size outside 0..65535, NULL strides for n > 1, negative stride
    assert lib.glu_apply_batched(-1, C.byref(bs), C.byref(th), C.byref(Tl), C.byref(p), C.byref(Th), None) == 4
    assert lib.glu_apply_batched(70000, C.byref(bs), C.byref(th), C.byref(Tl), C.byref(p), C.byref(Th), None) == 4
    assert lib.glu_apply_batched(2, None, C.byref(th), C.byref(Tl), C.byref(p), C.byref(Th), None) == 1
    neg = L.glu_batch_strides(64, -4, 64, 0, 0)
    assert lib.glu_apply_batched(2, C.byref(neg), C.byref(th), C.byref(Tl), C.byref(p), C.byref(Th), None) == 4
    # output images that overlap
    small = L.glu_batch_strides(64, 4, 8, 0, 0)
    assert lib.glu_apply_batched(2, C.byref(small), C.byref(th), C.byref(Tl), C.byref(p), C.byref(Th), None) == 2
    # an empty batch is valid and launches nothing
    assert lib.glu_apply_batched(0, None, C.byref(th), C.byref(Tl), C.byref(p), C.byref(Th), None) == 0
    G = _img(Cn=1)
    gT = _img(ptr=0x5000, H=2, W=2, Cn=1)
    ws = lib.glu_apply_backward_batched_workspace(3, 8, 8, 1, C.byref(p))
    assert ws == 3 * lib.glu_apply_backward_workspace(8, 8, 1, C.byref(p))
    bsb = L.glu_batch_strides(64, 4, 64, 1, 64)
    assert lib.glu_apply_backward_batched(3, C.byref(bsb), C.byref(th), C.byref(Tl), C.byref(p), C.byref(G),
                                          C.byref(gT), None, 0x6000, ws, None) == 2  # grad_T_low overlap
    bsb = L.glu_batch_strides(64, 4, 64, 4, 64)
    assert lib.glu_apply_backward_batched(3, C.byref(bsb), C.byref(th), C.byref(Tl), C.byref(p), C.byref(G),
                                          C.byref(gT), None, 0x6000, ws - 4, None) == 9  # workspace too small


def test_joint_downsample_grad_validation():
    lib = L.load()
    p = _params(s=4)
    I = _img(H=8, W=8)
    Il = _img(ptr=0x4000, H=2, W=2)
    th = _theta()
    ws = lib.glu_joint_downsample_grad_workspace(8, 8, C.byref(p))
    assert ws > 0

    def call(I=I, Il=Il, eta=0.01, n=2, wsp=0x100000, wsb=ws, err=0x7000):
        return lib.glu_joint_downsample_grad(C.byref(I), C.byref(Il), C.byref(p), eta, n, 1, C.byref(th), err, wsp,
                                             wsb, None, None, None)

    assert call(eta=-1.0) == 4
    assert call(eta=float("inf")) == 4
    assert call(n=65) == 4
    assert call(I=_img(H=8, W=8, dt=L.GLU_F16)) == 3
    assert call(Il=_img(ptr=0x4000, H=3, W=2)) == 2
    assert call(wsb=ws - 1) == 9
    assert call(wsp=0x100010) == 5
    # a non-dense theta needs a caller E buffer
    th2 = L.glu_theta(0x2000, 0x3000, 8, 8, 12)
    st = lib.glu_joint_downsample_grad(C.byref(I), C.byref(Il), C.byref(p), 0.01, 2, 1, C.byref(th2), None,
                                       0x100000, ws, None, None, None)
    assert st == 2


def test_joint_downsampling_rejects_flags():
    """The pairs-only candidate set (GLU_FLAG_NO_DEGENERATE) is a search
    option: both joint downsampling calls refuse it before any HIP call."""
    lib = L.load()
    p = _params(s=4, flags=L.GLU_FLAG_NO_DEGENERATE)
    I = _img(H=8, W=8)
    Il = _img(ptr=0x4000, H=2, W=2)
    th = _theta()
    ws = lib.glu_joint_downsample_grad_workspace(8, 8, C.byref(p))
    st = lib.glu_joint_downsample_grad(C.byref(I), C.byref(Il), C.byref(p), 0.01, 2, 1, C.byref(th), 0x7000,
                                       0x100000, ws, None, None, None)
    assert st == 8 and b"flags" in lib.glu_last_error()
    wsj = lib.glu_joint_downsample_workspace(8, 8, C.byref(p))
    st = lib.glu_joint_downsample(C.byref(I), C.byref(Il), C.byref(p), 30.0 / 255, 3, C.byref(th), 0x7000,
                                  0x100000, wsj, None, None, None)
    assert st == 8 and b"flags" in lib.glu_last_error()


def test_static_backward_rejects_sizes_beyond_its_array():
    """glu_apply_backward_static checks the workspace a call needs against its
    fixed array before any device call: too large is GLU_ERR_WORKSPACE."""
    lib = L.load()
    p = _params(s=1, k=3)
    H, W = 1024, 1024  # 1024^2 cells x 9 offsets x 3 channels x 4 bytes = 108 MiB
    need = lib.glu_apply_backward_workspace(H, W, 3, C.byref(p))
    assert need > L.GLU_STATIC_SCRATCH_BYTES
    th = L.glu_theta(0x1000, 0x2000, H, W, W)
    Tl = _img(ptr=0x3000, H=H, W=W, Cn=3)
    G = _img(ptr=0x4000, H=H, W=W, Cn=3)
    gT = _img(ptr=0x5000, H=H, W=W, Cn=3)
    st = lib.glu_apply_backward_static(C.byref(th), C.byref(Tl), C.byref(p), C.byref(G), C.byref(gT), None, None)
    assert st == 9, lib.glu_last_error()
    assert b"static array" in lib.glu_last_error()
    st = lib.glu_apply_backward_static(C.byref(th), C.byref(Tl), None, C.byref(G), C.byref(gT), None, None)
    assert st == 1
