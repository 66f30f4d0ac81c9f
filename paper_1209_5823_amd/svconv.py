"""Python binding of libsvconv (argument marshalling only).

Every computation runs in the HIP kernels behind the C ABI of
include/svconv.h; torch provides device memory and the stream.  Names follow
the C entry points: ``Plan.forward`` is ``svconv_forward`` and so on.

    plan = Plan(2048, 4096, 10, sigmas=(0.7, 1.5, 2.0), degrees=(6, 4, 2),
                spatial_degree=2, precision="fp32")
    D = plan.difference(R, I, a)          # D = (R (x) K(x,y)) - I  (Eq. 1)
"""

import ctypes

import torch

from . import _lib
from ._lib import check, PRECISIONS, FORMS


def _dev_ptr(t, dtype, shape, name):
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch tensor" % name)
    if t.device.type != "cuda":
        raise ValueError("%s must be on the GPU" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if tuple(t.shape) != tuple(shape):
        raise ValueError("%s must have shape %s, got %s" % (name, tuple(shape), tuple(t.shape)))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    return ctypes.c_void_p(t.data_ptr())


def _opt_ptr(t, dtype, shape, name):
    return None if t is None else _dev_ptr(t, dtype, shape, name)


class Plan:
    """An svconv plan: image size, kernel half-width, basis and spatial degree."""

    def __init__(self, height, width, half_width, sigmas, degrees, spatial_degree,
                 precision="fp32", form="basis", frame=None, pedestal=0.0):
        """Gaussian-basis plan; sigmas=None, degrees=None gives the Dirac delta
        basis (one basis per kernel pixel, see ``Plan.dfb``)."""
        self._lib = _lib.load()
        self._p = ctypes.c_void_p()
        if sigmas is None:
            check(self._lib.svconv_plan_create_dfb(ctypes.byref(self._p), int(height), int(width),
                                                   int(half_width), int(spatial_degree),
                                                   PRECISIONS[precision]),
                  "svconv_plan_create_dfb")
            sigmas, degrees = (), ()
        else:
            sig = (ctypes.c_double * len(sigmas))(*[float(s) for s in sigmas])
            deg = (ctypes.c_int * len(degrees))(*[int(d) for d in degrees])
            if len(sigmas) != len(degrees):
                raise ValueError("sigmas and degrees differ in length")
            check(self._lib.svconv_plan_create(ctypes.byref(self._p), int(height), int(width),
                                               int(half_width), len(sigmas), sig, deg,
                                               int(spatial_degree), PRECISIONS[precision]),
                  "svconv_plan_create")
        self.height, self.width, self.half_width = int(height), int(width), int(half_width)
        self.k = 2 * self.half_width + 1
        self.sigmas, self.degrees = tuple(sigmas), tuple(degrees)
        self.spatial_degree = int(spatial_degree)
        n, m = ctypes.c_int(), ctypes.c_int()
        check(self._lib.svconv_plan_sizes(self._p, ctypes.byref(n), ctypes.byref(m)), "sizes")
        self.n_basis, self.n_spatial = n.value, m.value
        self.precision, self.form = precision, "basis"
        self.background = False
        self.set_form(form)
        if frame is not None:
            self.set_frame(*frame)
        if pedestal:
            self.set_pedestal(pedestal)

    @classmethod
    def dfb(cls, height, width, half_width, spatial_degree, precision="fp32", form="regrouped",
            frame=None, pedestal=0.0):
        """Dirac delta basis plan (svconv_plan_create_dfb): a is [k*k][M]."""
        return cls(height, width, half_width, None, None, spatial_degree, precision=precision,
                   form=form, frame=frame, pedestal=pedestal)

    # ---------------------------------------------------------- settings --
    def set_frame(self, x0, y0, frame_width, frame_height):
        check(self._lib.svconv_plan_set_frame(self._p, int(x0), int(y0), int(frame_width),
                                              int(frame_height)), "svconv_plan_set_frame")

    def set_precision(self, precision):
        check(self._lib.svconv_plan_set_precision(self._p, PRECISIONS[precision]),
              "svconv_plan_set_precision")
        self.precision = precision

    def set_form(self, form):
        check(self._lib.svconv_plan_set_form(self._p, FORMS[form]), "svconv_plan_set_form")
        self.form = form

    def set_background(self, enable):
        """Fit model D = R (x) K + bg - I with bg = sum_m b_m P_m (the fit entry
        points then take (N + 1) x M coefficients: a, then b)."""
        check(self._lib.svconv_plan_set_background(self._p, 1 if enable else 0),
              "svconv_plan_set_background")
        self.background = bool(enable)

    def set_pedestal(self, pedestal):
        check(self._lib.svconv_plan_set_pedestal(self._p, float(pedestal)),
              "svconv_plan_set_pedestal")

    def basis(self):
        """float64 basis table B[n][v+h][u+h] as a CPU tensor."""
        out = torch.zeros((self.n_basis, self.k, self.k), dtype=torch.float64)
        check(self._lib.svconv_plan_get_basis(
            self._p, ctypes.cast(out.data_ptr(), ctypes.POINTER(ctypes.c_double))),
            "svconv_plan_get_basis")
        return out

    def _sync_stream(self):
        s = torch.cuda.current_stream().cuda_stream
        check(self._lib.svconv_plan_set_stream(self._p, ctypes.c_void_p(s)),
              "svconv_plan_set_stream")

    @property
    def _img(self):
        return (self.height, self.width)

    @property
    def _coef(self):
        return (self.n_basis, self.n_spatial)

    @property
    def _fit_coef(self):
        """Shape of the fit's coefficient arrays: a [N][M], plus b [M] with a
        background."""
        return (self.n_basis + (1 if self.background else 0), self.n_spatial)

    # ------------------------------------------------------------ compute --
    def forward(self, R, a, out=None):
        """out = R (x) K(x,y) (Eq. 1 without the subtraction)."""
        if out is None:
            out = torch.empty(self._img, dtype=torch.float32, device=R.device)
        self._sync_stream()
        check(self._lib.svconv_forward(self._p, _dev_ptr(R, torch.float32, self._img, "R"),
                                       _dev_ptr(a, torch.float32, self._coef, "a"),
                                       _dev_ptr(out, torch.float32, self._img, "out")),
              "svconv_forward")
        return out

    def difference(self, R, I, a, out=None):
        """D = (R (x) K(x,y)) - I (Eq. 1)."""
        if out is None:
            out = torch.empty(self._img, dtype=torch.float32, device=R.device)
        self._sync_stream()
        check(self._lib.svconv_difference(self._p, _dev_ptr(R, torch.float32, self._img, "R"),
                                          _dev_ptr(I, torch.float32, self._img, "I"),
                                          _dev_ptr(a, torch.float32, self._coef, "a"),
                                          _dev_ptr(out, torch.float32, self._img, "D")),
              "svconv_difference")
        return out

    def backward(self, R, a, gD, want_gR=True, want_ga=True):
        """(dL/dR float32, dL/da float64) for gD = dL/dD; either may be None."""
        gR = torch.empty(self._img, dtype=torch.float32, device=R.device) if want_gR else None
        ga = torch.empty(self._coef, dtype=torch.float64, device=R.device) if want_ga else None
        self._sync_stream()
        check(self._lib.svconv_backward(self._p, _dev_ptr(R, torch.float32, self._img, "R"),
                                        _dev_ptr(a, torch.float32, self._coef, "a"),
                                        _dev_ptr(gD, torch.float32, self._img, "gD"),
                                        _opt_ptr(gR, torch.float32, self._img, "gR"),
                                        _opt_ptr(ga, torch.float64, self._coef, "ga")),
              "svconv_backward")
        return gR, ga

    def loss_grad(self, D, mask=None, gD=None):
        """(L = sum_mask D^2 as a 0-d float64 tensor, gD = 2 D 1_mask)."""
        if gD is None:
            gD = torch.empty(self._img, dtype=torch.float32, device=D.device)
        loss = torch.empty((), dtype=torch.float64, device=D.device)
        self._sync_stream()
        check(self._lib.svconv_loss_grad(self._p, _dev_ptr(D, torch.float32, self._img, "D"),
                                         _opt_ptr(mask, torch.uint8, self._img, "mask"),
                                         _dev_ptr(gD, torch.float32, self._img, "gD"),
                                         _dev_ptr(loss, torch.float64, (), "loss")),
              "svconv_loss_grad")
        return loss, gD

    def normal_matrix(self, R, mask=None):
        """Phi^T Phi over the mask, Phi[p][(n,m)] = P_m(p) T_n(p); float64."""
        nm = self._fit_coef[0] * self._fit_coef[1]
        JtJ = torch.empty((nm, nm), dtype=torch.float64, device=R.device)
        self._sync_stream()
        check(self._lib.svconv_normal_matrix(self._p, _dev_ptr(R, torch.float32, self._img, "R"),
                                             _opt_ptr(mask, torch.uint8, self._img, "mask"),
                                             _dev_ptr(JtJ, torch.float64, (nm, nm), "JtJ")),
              "svconv_normal_matrix")
        return JtJ

    def normal_equations(self, R, I, mask=None):
        """(Phi^T Phi, Phi^T I) over the mask in one pass; float64."""
        nm = self._fit_coef[0] * self._fit_coef[1]
        JtJ = torch.empty((nm, nm), dtype=torch.float64, device=R.device)
        rhs = torch.empty((nm,), dtype=torch.float64, device=R.device)
        self._sync_stream()
        check(self._lib.svconv_normal_equations(self._p, _dev_ptr(R, torch.float32, self._img, "R"),
                                                _dev_ptr(I, torch.float32, self._img, "I"),
                                                _opt_ptr(mask, torch.uint8, self._img, "mask"),
                                                _dev_ptr(JtJ, torch.float64, (nm, nm), "JtJ"),
                                                _dev_ptr(rhs, torch.float64, (nm,), "rhs")),
              "svconv_normal_equations")
        return JtJ, rhs

    def cholesky_factor(self, A):
        """In-place Cholesky factor (lower) of a float64 SPD matrix."""
        n = A.shape[0]
        self._sync_stream()
        check(self._lib.svconv_cholesky_factor(self._p, _dev_ptr(A, torch.float64, (n, n), "A"),
                                               n), "svconv_cholesky_factor")
        return A

    def cholesky_solve(self, L, rhs, out=None):
        n = L.shape[0]
        if out is None:
            out = torch.empty((n,), dtype=torch.float64, device=L.device)
        self._sync_stream()
        check(self._lib.svconv_cholesky_solve(self._p, _dev_ptr(L, torch.float64, (n, n), "L"),
                                              _dev_ptr(rhs, torch.float64, (n,), "rhs"),
                                              _dev_ptr(out, torch.float64, (n,), "x"), n),
              "svconv_cholesky_solve")
        return out

    def gn_step(self, R, I, L, a64, a32, D, mask=None, stats=True):
        """One Gauss-Newton step; returns (loss before the step, ||delta||)."""
        fc = self._fit_coef
        nm = fc[0] * fc[1]
        st = (ctypes.c_double * 2)() if stats else None
        self._sync_stream()
        check(self._lib.svconv_gn_step(self._p, _dev_ptr(R, torch.float32, self._img, "R"),
                                       _dev_ptr(I, torch.float32, self._img, "I"),
                                       _opt_ptr(mask, torch.uint8, self._img, "mask"),
                                       _dev_ptr(L, torch.float64, (nm, nm), "L"),
                                       _dev_ptr(a64, torch.float64, fc, "a64"),
                                       _dev_ptr(a32, torch.float32, fc, "a32"),
                                       _dev_ptr(D, torch.float32, self._img, "D"), st),
              "svconv_gn_step")
        return (st[0], st[1]) if stats else None

    def ls_step(self, R, I, A, L, rhs, a64, a32, D, mask=None, stats=True):
        """One Newton step on the normal equations (A = JtJ, L its factor,
        rhs = J^T I); returns (loss before the step, ||delta||)."""
        fc = self._fit_coef
        nm = fc[0] * fc[1]
        st = (ctypes.c_double * 2)() if stats else None
        self._sync_stream()
        check(self._lib.svconv_ls_step(self._p, _dev_ptr(R, torch.float32, self._img, "R"),
                                       _dev_ptr(I, torch.float32, self._img, "I"),
                                       _opt_ptr(mask, torch.uint8, self._img, "mask"),
                                       _dev_ptr(A, torch.float64, (nm, nm), "A"),
                                       _dev_ptr(L, torch.float64, (nm, nm), "L"),
                                       _dev_ptr(rhs, torch.float64, (nm,), "rhs"),
                                       _dev_ptr(a64, torch.float64, fc, "a64"),
                                       _dev_ptr(a32, torch.float32, fc, "a32"),
                                       _dev_ptr(D, torch.float32, self._img, "D"), st),
              "svconv_ls_step")
        return (st[0], st[1]) if stats else None

    def pcg_fit(self, R, I, L, a64, a32, D, iters, mask=None, residuals=True):
        """Preconditioned conjugate gradients on the normal equations
        (svconv_pcg_fit); a64 is updated in place.  Returns the residual norm
        after each iteration (a list) when residuals=True."""
        fc = self._fit_coef
        nm = fc[0] * fc[1]
        res = (ctypes.c_double * max(int(iters), 1))() if residuals else None
        self._sync_stream()
        check(self._lib.svconv_pcg_fit(self._p, _dev_ptr(R, torch.float32, self._img, "R"),
                                       _dev_ptr(I, torch.float32, self._img, "I"),
                                       _opt_ptr(mask, torch.uint8, self._img, "mask"),
                                       _dev_ptr(L, torch.float64, (nm, nm), "L"), int(iters),
                                       _dev_ptr(a64, torch.float64, fc, "a64"),
                                       _dev_ptr(a32, torch.float32, fc, "a32"),
                                       _dev_ptr(D, torch.float32, self._img, "D"), res),
              "svconv_pcg_fit")
        return list(res)[:int(iters)] if residuals else None

    def stamp_mask(self, R, sky, threshold, frac=0.1, r_iso=None, margin=None, stamp_half=None,
                   mask=None):
        """Isolated-star stamp mask (svconv_stamp_mask); returns (mask, n_centres).
        Defaults: stamp_half = r_iso = the kernel half-width, margin = 2 h."""
        h = self.half_width
        r_iso = max(1, h) if r_iso is None else r_iso
        stamp_half = h if stamp_half is None else stamp_half
        margin = 2 * h if margin is None else margin
        if mask is None:
            mask = torch.empty(self._img, dtype=torch.uint8, device=R.device)
        n = ctypes.c_int(0)
        self._sync_stream()
        check(self._lib.svconv_stamp_mask(self._p, _dev_ptr(R, torch.float32, self._img, "R"),
                                          float(sky), float(threshold), float(frac), int(r_iso),
                                          int(margin), int(stamp_half),
                                          _dev_ptr(mask, torch.uint8, self._img, "mask"),
                                          ctypes.byref(n)), "svconv_stamp_mask")
        return mask, n.value

    def add_background(self, b, D):
        """D += sum_m b_m P_m (in place); b float32 [M] on the GPU."""
        self._sync_stream()
        check(self._lib.svconv_add_background(self._p, _dev_ptr(b, torch.float32,
                                                                (self.n_spatial,), "b"),
                                              _dev_ptr(D, torch.float32, self._img, "D")),
              "svconv_add_background")
        return D

    # ----------------------------------------------------------- lifetime --
    def close(self):
        if getattr(self, "_p", None) is not None and self._p.value:
            check(self._lib.svconv_plan_destroy(self._p), "svconv_plan_destroy")
            self._p = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def plan_for(workload, precision="fp32", form="basis", **kw):
    """Plan with the sizes and basis of a synth.Workload-like object."""
    return Plan(workload.height, workload.width, workload.half_width, workload.sigmas,
                workload.degrees, workload.spatial_degree, precision=precision, form=form, **kw)


class SVConvDifference(torch.autograd.Function):
    """D = (R (x) K(a)) - I with the hand-written adjoint as its backward.

    backward returns (dL/dR, dL/dI = -gD, dL/da cast to a's dtype).
    """

    @staticmethod
    def forward(ctx, plan, R, I, a):
        ctx.plan = plan
        ctx.save_for_backward(R, a)
        return plan.difference(R.detach().contiguous(), I.detach().contiguous(),
                               a.detach().contiguous())

    @staticmethod
    def backward(ctx, gD):
        plan = ctx.plan
        R, a = ctx.saved_tensors
        need_R, need_I, need_a = ctx.needs_input_grad[1], ctx.needs_input_grad[2], ctx.needs_input_grad[3]
        gD = gD.contiguous()
        gR, ga = None, None
        if need_R or need_a:
            gR, ga = plan.backward(R.detach().contiguous(), a.detach().contiguous(), gD,
                                   want_gR=need_R, want_ga=need_a)
        gI = torch.neg(gD) if need_I else None
        return None, gR, gI, (ga.to(a.dtype) if ga is not None else None)


def difference(plan, R, I, a):
    """Differentiable D = (R (x) K(a)) - I."""
    return SVConvDifference.apply(plan, R, I, a)


def difference_noalloc(R, I, a, half_width, sigmas, degrees, spatial_degree, precision="fp16x3",
                       pedestal=0.0, out=None):
    """D = (R (x) K(x,y)) - I without a plan and without any allocation in the
    library (svconv_difference_noalloc): the regrouped separable form, every
    table built on the device in the library's static scratch array, on
    torch's current stream.  R, I, out: float32 [H][W]; a: float32 [N][M]."""
    lib = _lib.load()
    H, W = R.shape
    if out is None:
        out = torch.empty((H, W), dtype=torch.float32, device=R.device)
    if len(sigmas) != len(degrees):
        raise ValueError("sigmas and degrees differ in length")
    N = sum((int(d) + 1) * (int(d) + 2) // 2 for d in degrees)
    M = (int(spatial_degree) + 1) * (int(spatial_degree) + 2) // 2
    sig = (ctypes.c_double * len(sigmas))(*[float(x) for x in sigmas])
    deg = (ctypes.c_int * len(degrees))(*[int(d) for d in degrees])
    s = torch.cuda.current_stream().cuda_stream
    check(lib.svconv_difference_noalloc(int(H), int(W), int(half_width), len(sigmas), sig, deg,
                                        int(spatial_degree), PRECISIONS[precision], float(pedestal),
                                        _dev_ptr(R, torch.float32, (H, W), "R"),
                                        _dev_ptr(I, torch.float32, (H, W), "I"),
                                        _dev_ptr(a, torch.float32, (N, M), "a"),
                                        _dev_ptr(out, torch.float32, (H, W), "D"), ctypes.c_void_p(s)),
          "svconv_difference_noalloc")
    return out


def _host_ptr(t, shape, name):
    """Address of a contiguous float32 CPU tensor or numpy array."""
    if isinstance(t, torch.Tensor):
        if t.device.type != "cpu":
            raise ValueError("%s must be in host memory" % name)
        if t.dtype != torch.float32:
            raise TypeError("%s must be float32, got %s" % (name, t.dtype))
        ok, addr, got = t.is_contiguous(), t.data_ptr(), tuple(t.shape)
    else:
        import numpy as np
        if not isinstance(t, np.ndarray) or t.dtype != np.float32:
            raise TypeError("%s must be a float32 tensor or array" % name)
        ok, addr, got = t.flags.c_contiguous, t.ctypes.data, t.shape
    if got != tuple(shape):
        raise ValueError("%s must have shape %s, got %s" % (name, tuple(shape), got))
    if not ok:
        raise ValueError("%s must be contiguous" % name)
    return addr


def pinned_empty(shape):
    """Page-locked float32 host tensor (the copies of a Pipeline overlap compute
    only from such memory)."""
    return torch.empty(shape, dtype=torch.float32, pin_memory=True)


class Pipeline:
    """Streamed difference images of host-resident tiles (svconv_pipeline_*):
    copies in, contraction and copies out of consecutive tiles overlap."""

    def __init__(self, plan, depth=3):
        self._lib = _lib.load()
        self.plan = plan
        self._q = ctypes.c_void_p()
        check(self._lib.svconv_pipeline_create(plan._p, int(depth), ctypes.byref(self._q)),
              "svconv_pipeline_create")

    def run(self, R_tiles, I_tiles, a_tiles, D_tiles):
        """D_tiles[t] = R_tiles[t] (x) K(a_tiles[t]) - I_tiles[t] for every t; all
        host float32 (pinned for overlap).  Blocks until every D is written."""
        n = len(R_tiles)
        if not (len(I_tiles) == len(a_tiles) == len(D_tiles) == n):
            raise ValueError("tile lists differ in length")
        img = (self.plan.height, self.plan.width)
        coef = (self.plan.n_basis, self.plan.n_spatial)
        arr = ctypes.c_void_p * max(n, 1)
        Rp = arr(*[_host_ptr(x, img, "R[%d]" % t) for t, x in enumerate(R_tiles)])
        Ip = arr(*[_host_ptr(x, img, "I[%d]" % t) for t, x in enumerate(I_tiles)])
        Ap = arr(*[_host_ptr(x, coef, "a[%d]" % t) for t, x in enumerate(a_tiles)])
        Dp = arr(*[_host_ptr(x, img, "D[%d]" % t) for t, x in enumerate(D_tiles)])
        check(self._lib.svconv_pipeline_run(self._q, n, Rp, Ip, Ap, Dp), "svconv_pipeline_run")

    def close(self):
        if getattr(self, "_q", None) is not None and self._q.value:
            check(self._lib.svconv_pipeline_destroy(self._q), "svconv_pipeline_destroy")
            self._q = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
