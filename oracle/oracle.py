"""Plain FP64 CPU oracle for spatially-varying-kernel image subtraction.

TEST INFRASTRUCTURE.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg import this module.  It wraps the plain C implementation in
``svconv_oracle.c`` (per-pixel kernel, direct convolution, in float64) and
adds one numpy routine, :func:`convolve_fft`, which evaluates the same
convolution through an exact regrouping of Eq. 2 (see its docstring) so that
large frames can be checked in seconds.  Nothing here is shared with the GPU
library, and nothing here imports it.

Every function takes the method's inputs explicitly: the reference image R,
the second image I, the coefficient array a[n][m] (n = basis, m = spatial
term), the kernel half-width h, the Gaussian widths and polynomial degrees
of the basis, the spatial degree and the frame (x0, y0, Wf, Hf) that fixes
the normalised coordinates.
"""

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "svconv_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)
_u8p = ctypes.POINTER(ctypes.c_ubyte)


def build(force=False):
    """Compile the C oracle with gcc (OpenMP) into ``liboracle.so``."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c99",
                           _SRC, "-o", tmp, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        i, d = ctypes.c_int, ctypes.c_double
        lib.orc_n_basis.argtypes = [i, _ip]
        lib.orc_n_spatial.argtypes = [i]
        lib.orc_basis.argtypes = [i, i, _dp, _ip, _dp]
        lib.orc_basis_dfb.argtypes = [i, _dp]
        lib.orc_spatial_terms.argtypes = [d, d, i, _dp]
        lib.orc_spatial_terms.restype = None
        lib.orc_kernel_at.argtypes = [i, i, i, i, _dp, i, _dp, i, i, i, i, _dp]
        lib.orc_convolve.argtypes = [i, i, _dp, i, i, _dp, i, _dp, i, i, i, i, _dp, i]
        lib.orc_convolve_at.argtypes = [i, i, _dp, i, i, _dp, i, _dp, i, i, i, i, i, _ip, _ip, _dp, i]
        lib.orc_grad_a.argtypes = [i, i, _dp, i, i, _dp, i, i, i, i, i, _dp, _dp, i]
        lib.orc_grad_R.argtypes = [i, i, i, i, _dp, i, _dp, i, i, i, i, _dp, _dp, i]
        lib.orc_normal_equations.argtypes = [i, i, _dp, _dp, i, i, _dp, i, i, i, i, i, _u8p, _dp, _dp]
        lib.orc_cholesky_solve.argtypes = [i, _dp, _dp, _dp]
        lib.orc_max_threads.argtypes = []
        _lib = lib
    return _lib


def _d(x):
    return np.ascontiguousarray(x, dtype=np.float64)


def _ptr(a, t=_dp):
    return a.ctypes.data_as(t)


def _check(rc, what):
    if rc < 0:
        raise ValueError("oracle %s failed with status %d" % (what, rc))
    return rc


def max_threads():
    return int(_load().orc_max_threads())


def n_basis(degrees):
    deg = np.ascontiguousarray(degrees, dtype=np.int32)
    return int(_load().orc_n_basis(len(deg), _ptr(deg, _ip)))


def n_spatial(d_s):
    return int(_load().orc_n_spatial(int(d_s)))


def basis(h, sigmas, degrees):
    """B[n][v+h][u+h] in float64 (Sec. 2, Eq. 2; unit L1 norm each)."""
    sig = _d(sigmas)
    deg = np.ascontiguousarray(degrees, dtype=np.int32)
    N = n_basis(deg)
    k = 2 * h + 1
    out = np.zeros((N, k, k))
    _check(_load().orc_basis(int(h), len(sig), _ptr(sig), _ptr(deg, _ip), _ptr(out)), "basis")
    return out


def basis_dfb(h):
    """Dirac delta basis: k*k bases, B[n] = 1 at n = (v+h) k + (u+h) (Sec. 2)."""
    k = 2 * h + 1
    out = np.zeros((k * k, k, k))
    _check(_load().orc_basis_dfb(int(h), _ptr(out)), "basis_dfb")
    return out


def spatial_terms(xh, yh, d_s):
    """P_m at one normalised position (Eq. 3 generalised to degree d_s)."""
    P = np.zeros(n_spatial(d_s))
    _load().orc_spatial_terms(float(xh), float(yh), int(d_s), _ptr(P))
    return P


def kernel_at(x, y, h, B, d_s, a, frame):
    """K(x,y)[v+h][u+h] at one array pixel (Eq. 2)."""
    B = _d(B); a = _d(a)
    k = 2 * h + 1
    K = np.zeros((k, k))
    x0, y0, Wf, Hf = frame
    _check(_load().orc_kernel_at(int(x), int(y), int(h), B.shape[0], _ptr(B), int(d_s), _ptr(a),
                                 int(x0), int(y0), int(Wf), int(Hf), _ptr(K)), "kernel_at")
    return K


def _frame(frame, R):
    if frame is None:
        return (0, 0, R.shape[1], R.shape[0])
    return tuple(int(v) for v in frame)


def convolve(R, h, B, d_s, a, frame=None, nthreads=0):
    """C = R (x) K(x,y): per-pixel kernel, direct convolution, float64."""
    R = _d(R); B = _d(B); a = _d(a)
    H, W = R.shape
    x0, y0, Wf, Hf = _frame(frame, R)
    C = np.zeros((H, W))
    _check(_load().orc_convolve(H, W, _ptr(R), int(h), B.shape[0], _ptr(B), int(d_s), _ptr(a),
                                x0, y0, Wf, Hf, _ptr(C), int(nthreads)), "convolve")
    return C


def difference(R, I, h, B, d_s, a, frame=None, nthreads=0):
    """D = (R (x) K(x,y)) - I (Eq. 1), float64."""
    return convolve(R, h, B, d_s, a, frame, nthreads) - _d(I)


def convolve_at(R, h, B, d_s, a, xs, ys, frame=None, nthreads=0):
    """C at the array pixels (xs[i], ys[i]) only."""
    R = _d(R); B = _d(B); a = _d(a)
    H, W = R.shape
    xs = np.ascontiguousarray(xs, dtype=np.int32)
    ys = np.ascontiguousarray(ys, dtype=np.int32)
    x0, y0, Wf, Hf = _frame(frame, R)
    out = np.zeros(len(xs))
    _check(_load().orc_convolve_at(H, W, _ptr(R), int(h), B.shape[0], _ptr(B), int(d_s), _ptr(a),
                                   x0, y0, Wf, Hf, len(xs), _ptr(xs, _ip), _ptr(ys, _ip), _ptr(out),
                                   int(nthreads)), "convolve_at")
    return out


def interior_mask(H, W, h):
    """Omega: pixels at least h from every edge (the loss region)."""
    m = np.zeros((H, W), dtype=bool)
    if H > 2 * h and W > 2 * h:
        m[h:H - h, h:W - h] = True
    return m


def grad_a(R, h, B, d_s, G, frame=None, nthreads=0):
    """dL/da[n][m] = sum_p G(p) P_m(p) T_n(p) for G = dL/dD."""
    R = _d(R); B = _d(B); G = _d(G)
    H, W = R.shape
    x0, y0, Wf, Hf = _frame(frame, R)
    ga = np.zeros((B.shape[0], n_spatial(d_s)))
    _check(_load().orc_grad_a(H, W, _ptr(R), int(h), B.shape[0], _ptr(B), int(d_s),
                              x0, y0, Wf, Hf, _ptr(G), _ptr(ga), int(nthreads)), "grad_a")
    return ga


def grad_R(shape, h, B, d_s, a, G, frame=None, nthreads=0):
    """dL/dR(q) = sum_{u,v} G(q+(u,v)) K(q+(u,v))[u,v] for G = dL/dD."""
    B = _d(B); a = _d(a); G = _d(G)
    H, W = shape
    x0, y0, Wf, Hf = frame if frame is not None else (0, 0, W, H)
    gR = np.zeros((H, W))
    _check(_load().orc_grad_R(H, W, int(h), B.shape[0], _ptr(B), int(d_s), _ptr(a),
                              int(x0), int(y0), int(Wf), int(Hf), _ptr(G), _ptr(gR), int(nthreads)),
           "grad_R")
    return gR


def normal_equations(R, I, h, B, d_s, mask=None, frame=None):
    """(Phi^T Phi, Phi^T I) with Phi[p][(n,m)] = P_m(p) T_n(p) over the mask."""
    R = _d(R); B = _d(B)
    H, W = R.shape
    x0, y0, Wf, Hf = _frame(frame, R)
    NM = B.shape[0] * n_spatial(d_s)
    JtJ = np.zeros((NM, NM))
    rhs = np.zeros(NM)
    Ip = _d(I) if I is not None else None
    mk = np.ascontiguousarray(mask, dtype=np.uint8) if mask is not None else None
    _check(_load().orc_normal_equations(H, W, _ptr(R), _ptr(Ip) if Ip is not None else None,
                                        int(h), B.shape[0], _ptr(B), int(d_s), x0, y0, Wf, Hf,
                                        _ptr(mk, _u8p) if mk is not None else None,
                                        _ptr(JtJ), _ptr(rhs)), "normal_equations")
    return JtJ, rhs


def cholesky_solve(A, b):
    """x = A^-1 b for SPD A through A = L L^T; raises on a non-SPD matrix."""
    A = _d(A); b = _d(b)
    n = A.shape[0]
    x = np.zeros(n)
    rc = _load().orc_cholesky_solve(n, _ptr(A), _ptr(b), _ptr(x))
    if rc == -5:
        raise np.linalg.LinAlgError("matrix is not symmetric positive definite")
    _check(rc, "cholesky_solve")
    return x


def fit_least_squares(R, I, h, B, d_s, mask=None, frame=None):
    """Coefficients minimising sum_mask D^2 (OIS least squares, Sec. 2)."""
    JtJ, rhs = normal_equations(R, I, h, B, d_s, mask, frame)
    return cholesky_solve(JtJ, rhs).reshape(B.shape[0], n_spatial(d_s))


# ---------------------------------------------------------------------------
# Exact regrouping for large frames.
#
# Because the spatial terms P_m depend only on the output pixel, Eq. 2 can be
# regrouped as K(x,y) = sum_m P_m(x,y) Kt_m with Kt_m = sum_n a[n][m] B_n, so
# R (x) K(x,y) = sum_m P_m * (R (x) Kt_m): M ordinary (spatially constant)
# convolutions, each done here by zero-padded FFT.  This is the same value as
# the per-pixel form up to rounding, not an approximation.
# ---------------------------------------------------------------------------

def _fft_shape(H, W, k):
    from scipy import fft as sfft
    return sfft.next_fast_len(H + k - 1, real=True), sfft.next_fast_len(W + k - 1, real=True)


def _fft_conv_same(R, K, FR=None, shape=None, workers=-1):
    """Zero-padded linear convolution of R with a (k x k) kernel centred at h.

    FR (the transform of R at `shape`) may be passed to reuse it."""
    from scipy import fft as sfft
    H, W = R.shape
    k = K.shape[0]
    h = k // 2
    if shape is None:
        shape = _fft_shape(H, W, k)
    if FR is None:
        FR = sfft.rfft2(R, s=shape, workers=workers)
    full = sfft.irfft2(FR * sfft.rfft2(K, s=shape, workers=workers), s=shape, workers=workers)
    return full[h:h + H, h:h + W]


def convolve_fft(R, h, B, d_s, a, frame=None):
    """R (x) K(x,y) through the regrouping above; float64."""
    from scipy import fft as sfft
    R = _d(R); B = _d(B); a = _d(a)
    shape = _fft_shape(R.shape[0], R.shape[1], B.shape[1])
    FR = sfft.rfft2(R, s=shape, workers=-1)
    C = np.zeros(R.shape)
    M = n_spatial(d_s)
    x0, y0, Wf, Hf = frame if frame is not None else (0, 0, R.shape[1], R.shape[0])
    xs = np.arange(R.shape[1], dtype=np.float64) + x0
    ys = np.arange(R.shape[0], dtype=np.float64) + y0
    xh = 2.0 * xs / (Wf - 1) - 1.0 if Wf > 1 else 0.0 * xs
    yh = 2.0 * ys / (Hf - 1) - 1.0 if Hf > 1 else 0.0 * ys
    m = 0
    for t in range(d_s + 1):
        for i in range(t, -1, -1):
            Kt = np.tensordot(a[:, m], B, axes=(0, 0))
            conv = _fft_conv_same(R, Kt, FR, shape)
            C += conv * (yh ** (t - i))[:, None] * (xh ** i)[None, :]
            m += 1
    assert m == M
    return C


# ---------------------------------------------------------------------------
# Optimal Image Subtraction on isolated-star stamps (Sec. 2: isolated stars of
# the reference are the source the kernel is determined from), with a
# differential background polynomial.
#
# Readings taken here (the paper gives no numbers for them):
#   * a stamp centre is a pixel p whose value is strictly larger than each of
#     its (up to 8) neighbours inside the image, with R(p) - sky > threshold,
#     at least `margin` pixels from every edge, and with no other such local
#     maximum q within the (2 r_iso + 1)^2 window around p (clipped to the
#     image) for which R(q) - sky >= frac (R(p) - sky): a star is isolated
#     when no neighbour of comparable brightness is near it.  Every decision
#     is taken on float64 values of the float32 image.
#   * the stamp mask is the union of the (2 s + 1)^2 boxes around the centres.
#   * the background is bg(p) = sum_m b[m] P_m(p) with the spatial terms of
#     Eq. 3 (same degree as the kernel's), and the model is
#     D = (R (x) K) + bg - I.
# ---------------------------------------------------------------------------

def _strict_local_max(R64):
    H, W = R64.shape
    lmax = np.ones((H, W), dtype=bool)
    pad = np.full((H + 2, W + 2), -np.inf)
    pad[1:H + 1, 1:W + 1] = R64
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            if dx == 0 and dy == 0:
                continue
            lmax &= R64 > pad[1 + dy:1 + dy + H, 1 + dx:1 + dx + W]
    return lmax


def stamp_centres(R, sky, threshold, frac, r_iso, margin):
    """[(x, y), ...] of isolated-star stamp centres in raster order."""
    R64 = np.asarray(R, dtype=np.float64)
    H, W = R64.shape
    lmax = _strict_local_max(R64)
    cand = lmax & (R64 - sky > threshold)
    out = []
    for y, x in np.argwhere(cand):          # raster order
        if x < margin or x > W - 1 - margin or y < margin or y > H - 1 - margin:
            continue
        f = R64[y, x] - sky
        ok = True
        for qy in range(max(0, y - r_iso), min(H, y + r_iso + 1)):
            for qx in range(max(0, x - r_iso), min(W, x + r_iso + 1)):
                if (qx, qy) != (x, y) and lmax[qy, qx] and R64[qy, qx] - sky >= frac * f:
                    ok = False
        if ok:
            out.append((int(x), int(y)))
    return out


def stamp_mask(H, W, centres, s):
    """uint8 mask: 1 inside the (2 s + 1)^2 box of any centre."""
    m = np.zeros((H, W), dtype=np.uint8)
    for (x, y) in centres:
        m[max(0, y - s):min(H, y + s + 1), max(0, x - s):min(W, x + s + 1)] = 1
    return m


def spatial_term_images(H, W, d_s, frame=None):
    """P[m][y][x] at every array pixel (one orc_spatial_terms call each)."""
    x0, y0, Wf, Hf = frame if frame is not None else (0, 0, W, H)
    lib = _load()
    M = n_spatial(d_s)
    P = np.zeros((M, H, W))
    row = np.zeros(M)
    for y in range(H):
        yh = 2.0 * (y + y0) / (Hf - 1) - 1.0 if Hf > 1 else 0.0
        for x in range(W):
            xh = 2.0 * (x + x0) / (Wf - 1) - 1.0 if Wf > 1 else 0.0
            lib.orc_spatial_terms(xh, yh, int(d_s), _ptr(row))
            P[:, y, x] = row
    return P


def background(H, W, d_s, b, frame=None):
    """bg(p) = sum_m b[m] P_m(p)."""
    return np.tensordot(_d(b), spatial_term_images(H, W, d_s, frame), axes=(0, 0))


def basis_responses(R, h, B, frame=None):
    """T_n = B_n (x) R for every basis (the convolution with a = e_(n,0), P_0 = 1)."""
    R = _d(R); B = _d(B)
    N = B.shape[0]
    T = np.zeros((N,) + R.shape)
    for n in range(N):
        a = np.zeros((N, 1))
        a[n, 0] = 1.0
        T[n] = convolve(R, h, B, 0, a, frame)
    return T


def design_matrix_bg(R, h, B, d_s, mask=None, frame=None):
    """Phi[p][(n,m)] = P_m(p) T_n(p) for n < N and Phi[p][N M + m] = P_m(p),
    over the masked pixels (interior if mask is None), rows in raster order."""
    R = _d(R)
    H, W = R.shape
    T = basis_responses(R, h, B, frame)
    P = spatial_term_images(H, W, d_s, frame)
    sel = interior_mask(H, W, h) if mask is None else np.asarray(mask, dtype=bool)
    N, M = T.shape[0], P.shape[0]
    cols = [P[m][sel] * T[n][sel] for n in range(N) for m in range(M)]
    cols += [P[m][sel] for m in range(M)]
    return np.stack(cols, axis=1), sel


def normal_equations_bg(R, I, h, B, d_s, mask=None, frame=None):
    """(Phi^T Phi, Phi^T I) of the model with the background polynomial."""
    Phi, sel = design_matrix_bg(R, h, B, d_s, mask, frame)
    return Phi.T @ Phi, Phi.T @ _d(I)[sel]


def fit_least_squares_bg(R, I, h, B, d_s, mask=None, frame=None):
    """(a[N][M], b[M]) minimising sum_mask (R (x) K + bg - I)^2."""
    JtJ, rhs = normal_equations_bg(R, I, h, B, d_s, mask, frame)
    x = cholesky_solve(JtJ, rhs)
    N, M = _d(B).shape[0], n_spatial(d_s)
    return x[:N * M].reshape(N, M), x[N * M:]
