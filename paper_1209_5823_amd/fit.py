"""Gauss-Newton fit of the spatial coefficients a[n][m] (the least-squares
kernel fit of Optimal Image Subtraction, Sec. 2) on the GPU.

Every step runs in libsvconv: the float64 normal matrix and its Cholesky
factor once, then per iteration the forward difference (any precision), the
loss gradient, the adjoint in a, the two triangular solves and the update
(``svconv_gn_step``).  D is linear in a, so one exact step reaches the
least-squares solution; later steps refine it against the rounding of the
forward pass.
"""

import time

import torch


def gauss_newton_fit(plan, R, I, a0, iters=4, mask=None, timings=False):
    """Fit a starting from a0 (float32/64 [N][M] on the GPU).

    Returns (a64, D, history) with history rows (loss before the step,
    ||delta||, seconds for the step when timings=True).
    """
    t0 = time.perf_counter()
    JtJ = plan.normal_matrix(R, mask)
    plan.cholesky_factor(JtJ)          # synchronises the plan's stream
    t_setup = time.perf_counter() - t0
    a64 = a0.to(torch.float64).contiguous().clone()
    a32 = torch.empty(a64.shape, dtype=torch.float32, device=a64.device)
    D = torch.empty_like(R)
    hist = []
    for _ in range(iters):
        t = time.perf_counter()
        loss, step = plan.gn_step(R, I, JtJ, a64, a32, D, mask)   # synchronises
        hist.append((loss, step, time.perf_counter() - t if timings else None))
    # residual at the final coefficients
    a32.copy_(a64.to(torch.float32))
    plan.difference(R, I, a32, out=D)
    return a64, D, hist, t_setup
