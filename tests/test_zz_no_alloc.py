"""GPU check of glu_apply_backward_static, the allocation-free backward:
through the C ABI it gives bitwise the results of glu_apply_backward (which
takes a caller workspace) on two calls in a row, the second smaller than
the first (the library's array keeps the first call's contents), and it
refuses a call whose workspace would exceed its array."""
import numpy as np
import pytest
import torch

import oracle as O
import synth
from tests.gpu_util import dev, log_case, need_gpu

pytestmark = pytest.mark.gpu


def _case(glu, H, W, s, k, C, seed):
    I = synth.voronoi(H, W, n_cells=max(8, H * W // 20000), n_dots=8, dot_px=(1, 3), seed=seed)
    L = O.downsample_point(I, s)
    T = np.ascontiguousarray(synth.lr_op_f1(L)[..., :C].astype(np.float32))
    th = glu.search(dev(I), dev(L), s, k)
    g = torch.Generator(device="cuda")
    g.manual_seed(seed + 1)
    G = torch.randn((H, W, C), generator=g, device="cuda")
    return th, dev(T), G


def test_static_backward_matches_workspace_backward():
    need_gpu()
    import paper_2307_09582_amd as glu

    for H, W, s, k, C, seed in ((2160, 3840, 8, 3, 3, 41), (333, 517, 4, 5, 1, 42)):
        log_case(test="no_alloc_backward", H=H, W=W, s=s, k=k, C=C)
        th, T, G = _case(glu, H, W, s, k, C, seed)
        ref_T, ref_a = glu.apply_backward(th, T, G, s, k)
        got_T, got_a = glu.apply_backward_static(th, T, G, s, k)
        torch.cuda.synchronize()
        assert torch.equal(got_T, ref_T) and torch.equal(got_a, ref_a)
        # the gradient with respect to T_low alone, and dalpha alone
        got_T2, none_a = glu.apply_backward_static(th, T, G, s, k, need_alpha=False)
        none_T, got_a2 = glu.apply_backward_static(th, T, G, s, k, need_T_low=False)
        torch.cuda.synchronize()
        assert none_a is None and none_T is None
        assert torch.equal(got_T2, ref_T) and torch.equal(got_a2, ref_a)


def test_static_backward_refuses_beyond_its_array():
    need_gpu()
    import paper_2307_09582_amd as glu
    from paper_2307_09582_amd import _lib as L

    H, W, s = 1024, 1024, 1
    assert glu.apply_backward_workspace(H, W, 3, s, 3) > L.GLU_STATIC_SCRATCH_BYTES
    th = glu.empty_theta(H, W)
    T = torch.zeros((H, W, 3), device="cuda")
    G = torch.zeros((H, W, 3), device="cuda")
    with pytest.raises(L.GluError) as ei:
        glu.apply_backward_static(th, T, G, s, 3)
    assert ei.value.name == "GLU_ERR_WORKSPACE"
