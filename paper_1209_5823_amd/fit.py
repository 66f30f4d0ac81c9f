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


def _final_residual(plan, R, I, a64, a32, D):
    """D at the final coefficients (with the background polynomial, when the
    plan fits one, in the last row of a)."""
    a32.copy_(a64.to(torch.float32))
    N = plan.n_basis
    if a32.shape[0] > N:
        plan.difference(R, I, a32[:N].contiguous(), out=D)
        plan.add_background(a32[N].contiguous(), D)
    else:
        plan.difference(R, I, a32, out=D)


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
    _final_residual(plan, R, I, a64, a32, D)
    return a64, D, hist, t_setup


def least_squares_fit(plan, R, I, a0, iters=3, mask=None, timings=False):
    """Fit a from a0 on the normal equations (JtJ, J^T I) built in one pass:
    each iteration forms D and its loss at the current a, then the float64
    Newton step (JtJ)^-1 (JtJ a - J^T I).  Same returns as gauss_newton_fit.
    """
    t0 = time.perf_counter()
    A, rhs = plan.normal_equations(R, I, mask)
    L = A.clone()
    plan.cholesky_factor(L)            # synchronises the plan's stream
    t_setup = time.perf_counter() - t0
    a64 = a0.to(torch.float64).contiguous().clone()
    a32 = torch.empty(a64.shape, dtype=torch.float32, device=a64.device)
    D = torch.empty_like(R)
    hist = []
    for _ in range(iters):
        t = time.perf_counter()
        loss, step = plan.ls_step(R, I, A, L, rhs, a64, a32, D, mask)   # synchronises
        hist.append((loss, step, time.perf_counter() - t if timings else None))
    _final_residual(plan, R, I, a64, a32, D)
    return a64, D, hist, t_setup


def stamp_preconditioned_fit(plan, R, I, a0, sky, threshold, frac=0.1, iters=8, mask=None,
                             stamp_iters=1, rounds=1, timings=False):
    """Optimal Image Subtraction on isolated stars, then the whole image.

    1. stamp mask of the isolated stars of R (svconv_stamp_mask);
    2. normal matrix of the stamps and its Cholesky factor;
    3. Gauss-Newton on the stamps from a0 (one step is the stamp solution);
    4. conjugate gradients on the whole image's normal equations (over
       `mask`, default the interior) from the stamp solution, preconditioned
       by the stamp factor (svconv_pcg_fit), in `rounds` calls of `iters`
       iterations; each call restarts from the true residual.

    a0 is float32/64 [N][M] (or [N+1][M] with the plan's background on).
    Returns (a64, D, info); info holds n_centres, the stamp coverage, the
    residual norm after each CG iteration and, with timings, the seconds of
    each phase.
    """
    info = {}
    t0 = time.perf_counter()
    smask, n_c = plan.stamp_mask(R, sky, threshold, frac)   # synchronises
    info["n_centres"] = n_c
    info["stamp_fraction"] = float(smask.float().mean().item())
    t1 = time.perf_counter()
    JtJ = plan.normal_matrix(R, smask)
    plan.cholesky_factor(JtJ)                                 # synchronises
    t2 = time.perf_counter()
    a64 = a0.to(torch.float64).contiguous().clone()
    a32 = torch.empty(a64.shape, dtype=torch.float32, device=a64.device)
    D = torch.empty_like(R)
    for _ in range(stamp_iters):
        plan.gn_step(R, I, JtJ, a64, a32, D, smask)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    info["a_stamps"] = a64.clone()
    info["residuals"] = []
    for _ in range(rounds):
        info["residuals"] += plan.pcg_fit(R, I, JtJ, a64, a32, D, iters, mask)   # synchronises
    t4 = time.perf_counter()
    if timings:
        info["t_stamps"] = t1 - t0
        info["t_stamp_normal"] = t2 - t1
        info["t_stamp_fit"] = t3 - t2
        info["t_pcg"] = t4 - t3
    return a64, D, info
