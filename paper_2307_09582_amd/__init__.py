"""Guided linear upsampling (Song et al., ACM TOG 2023) on AMD MI355X.

The hot path (pair search, apply, its backward, joint downsampling and
batched execution) runs in HIP kernels for gfx950 behind the C ABI of
include/glu.h; this package is the thin torch binding over it.
"""
from .glu import (  # noqa: F401
    EPS,
    N_ITER,
    TAU,
    BatchPlan,
    GluApply,
    Theta,
    autotune,
    autotune_load,
    autotune_save,
    apply,
    apply_backward,
    apply_backward_static,
    apply_backward_workspace,
    apply_backward_batched_workspace,
    downsample,
    empty_theta,
    glu_apply_autograd,
    joint_downsample,
    joint_downsample_grad,
    joint_downsample_workspace,
    lr_shape,
    search,
    search_apply,
    theta_expand,
)
from ._lib import GluError  # noqa: F401
