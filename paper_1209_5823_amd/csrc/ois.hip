// Optimal Image Subtraction on isolated stars (Sec. 2: the kernel is
// determined by least squares from isolated stars of the reference):
//   * stamp selection: isolated local maxima of R above a threshold, and the
//     mask of the boxes around them;
//   * the differential background polynomial bg = sum_m b_m P_m of the fit
//     model D = (R (x) K) + bg - I, and its gradient;
//   * the whole-image fit by conjugate gradients on the normal equations,
//     preconditioned by a Cholesky factor (typically that of the stamp normal
//     matrix, which is far cheaper to build than the whole-image one).
#include <cmath>

#include "internal.hpp"

namespace svc {

// ---------------------------------------------------------- stamps ----

// R(x,y) strictly larger than each of its neighbours inside the image.
__device__ __forceinline__ bool strict_local_max(const float* __restrict__ R, int H, int W, int x,
                                                 int y) {
    const float v = R[(size_t)y * W + x];
    for (int dy = -1; dy <= 1; ++dy) {
        const int ny = y + dy;
        if (ny < 0 || ny >= H) continue;
        for (int dx = -1; dx <= 1; ++dx) {
            const int nx = x + dx;
            if ((dx == 0 && dy == 0) || nx < 0 || nx >= W) continue;
            if (!(v > R[(size_t)ny * W + nx])) return false;
        }
    }
    return true;
}

// flags[p] = 1 for a stamp centre: a strict local maximum with R - sky >
// threshold, at least `margin` from every edge, and no other strict local
// maximum q in the (2 r_iso + 1)^2 window with R(q) - sky >= frac (R(p) - sky).
// Every comparison is taken in float64 on the float32 values.
__global__ void centre_kernel(const float* __restrict__ R, int H, int W, double sky, double thr,
                              double frac, int r_iso, int margin, unsigned char* __restrict__ flags) {
    const size_t n = (size_t)H * W;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const int y = (int)(i / W), x = (int)(i - (size_t)y * W);
        unsigned char f = 0;
        if (x >= margin && x <= W - 1 - margin && y >= margin && y <= H - 1 - margin) {
            const double v = (double)R[i] - sky;
            if (v > thr && strict_local_max(R, H, W, x, y)) {
                const double lim = frac * v;
                bool ok = true;
                const int y0 = max(0, y - r_iso), y1 = min(H - 1, y + r_iso);
                const int x0 = max(0, x - r_iso), x1 = min(W - 1, x + r_iso);
                for (int qy = y0; qy <= y1 && ok; ++qy)
                    for (int qx = x0; qx <= x1; ++qx) {
                        if (qx == x && qy == y) continue;
                        if ((double)R[(size_t)qy * W + qx] - sky >= lim &&
                            strict_local_max(R, H, W, qx, qy)) {
                            ok = false;
                            break;
                        }
                    }
                f = ok ? 1 : 0;
            }
        }
        flags[i] = f;
    }
}

// out[y][x] = max over |dx| <= s (rows) or |dy| <= s (columns) of in
__global__ void dilate_rows_kernel(const unsigned char* __restrict__ in, int H, int W, int s,
                                   unsigned char* __restrict__ out) {
    const size_t n = (size_t)H * W;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const int y = (int)(i / W), x = (int)(i - (size_t)y * W);
        const unsigned char* row = in + (size_t)y * W;
        unsigned char any = 0;
        for (int xx = max(0, x - s); xx <= min(W - 1, x + s); ++xx) any |= row[xx];
        out[i] = any;
    }
}

__global__ void dilate_cols_kernel(const unsigned char* __restrict__ in, int H, int W, int s,
                                   unsigned char* __restrict__ out) {
    const size_t n = (size_t)H * W;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const int y = (int)(i / W), x = (int)(i - (size_t)y * W);
        unsigned char any = 0;
        for (int yy = max(0, y - s); yy <= min(H - 1, y + s); ++yy) any |= in[(size_t)yy * W + x];
        out[i] = any;
    }
}

constexpr int COUNT_BLOCKS = 256;

// part[block] = number of set flags in the block's pixels; part[COUNT_BLOCKS]
// = their total (second kernel, fixed order)
__global__ void count_kernel(const unsigned char* __restrict__ flags, size_t n, int* __restrict__ part) {
    __shared__ int red[256];
    int c = 0;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        c += flags[i] ? 1 : 0;
    red[threadIdx.x] = c;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void count_total_kernel(int* __restrict__ part) {
    if (threadIdx.x == 0) {
        int t = 0;
        for (int b = 0; b < COUNT_BLOCKS; ++b) t += part[b];
        part[COUNT_BLOCKS] = t;
    }
}

// ------------------------------------------------------ background ----

__device__ __forceinline__ double ipow_d(double x, int e) {
    double r = 1.0;
    for (int t = 0; t < e; ++t) r *= x;
    return r;
}

// D += sum_m b_m P_m, P_m = xh^i yh^j in the order t = 0..d_s, i = t..0 (Eq. 3)
__global__ void add_background_kernel(float* __restrict__ D, const float* __restrict__ b, int H,
                                      int W, int d_s, double sx, double ox, double sy, double oy) {
    const size_t n = (size_t)H * W;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const int y = (int)(i / W), x = (int)(i - (size_t)y * W);
        const double xh = sx * x + ox, yh = sy * y + oy;
        double bg = 0.0;
        int m = 0;
        for (int t = 0; t <= d_s; ++t)
            for (int e = t; e >= 0; --e) bg += (double)b[m++] * ipow_d(xh, e) * ipow_d(yh, t - e);
        D[i] = (float)((double)D[i] + bg);
    }
}

constexpr int BG_BLOCKS = 64;

// part[block][m] = sum over the block's pixels of G P_m
__global__ __launch_bounds__(256) void bg_grad_kernel(const float* __restrict__ G, int H, int W,
                                                      int d_s, double sx, double ox, double sy,
                                                      double oy, double* __restrict__ part) {
    const int M = (d_s + 1) * (d_s + 2) / 2;
    double s[kMaxSpatialTerms];
#pragma unroll
    for (int m = 0; m < kMaxSpatialTerms; ++m) s[m] = 0.0;
    const size_t n = (size_t)H * W;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const float g = G[i];
        if (g == 0.f) continue;
        const int y = (int)(i / W), x = (int)(i - (size_t)y * W);
        const double xh = sx * x + ox, yh = sy * y + oy;
        int m = 0;
#pragma unroll
        for (int t = 0; t <= kMaxSpatialDegree; ++t)
#pragma unroll
            for (int e = t; e >= 0; --e) {
                if (t <= d_s) s[m] += (double)g * ipow_d(xh, e) * ipow_d(yh, t - e);
                ++m;
            }
    }
    __shared__ double red[256];
    // terms are numbered per degree, so term m of degree d_s sits at the same
    // index in the full (degree kMaxSpatialDegree) numbering
#pragma unroll
    for (int m = 0; m < kMaxSpatialTerms; ++m) {
        if (m < M) {   // uniform over the workgroup
            red[threadIdx.x] = s[m];
            __syncthreads();
            for (int o = 128; o > 0; o >>= 1) {
                if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
                __syncthreads();
            }
            if (threadIdx.x == 0) part[blockIdx.x * M + m] = red[0];
            __syncthreads();
        }
    }
}

__global__ void bg_grad_final(const double* __restrict__ part, int M, double* __restrict__ gb) {
    const int m = threadIdx.x;
    if (m >= M) return;
    double s = 0.0;
    for (int b = 0; b < BG_BLOCKS; ++b) s += part[b * M + m];
    gb[m] = s;
}

static void frame_coords(const svconv_plan* p, double& sx, double& ox, double& sy, double& oy) {
    sx = ox = sy = oy = 0.0;
    if (p->Wf > 1) { sx = 2.0 / (p->Wf - 1); ox = sx * p->x0 - 1.0; }
    if (p->Hf > 1) { sy = 2.0 / (p->Hf - 1); oy = sy * p->y0 - 1.0; }
}

int launch_add_background(svconv_plan* p, const float* b, float* D) {
    double sx, ox, sy, oy;
    frame_coords(p, sx, ox, sy, oy);
    hipLaunchKernelGGL(add_background_kernel, dim3(2048), dim3(256), 0, p->stream, D, b, p->H, p->W,
                       p->d_s, sx, ox, sy, oy);
    return hip_status(hipGetLastError(), "add_background_kernel");
}

int launch_bg_grad(svconv_plan* p, const float* G, double* gb) {
    double sx, ox, sy, oy;
    frame_coords(p, sx, ox, sy, oy);
    hipLaunchKernelGGL(bg_grad_kernel, dim3(BG_BLOCKS), dim3(256), 0, p->stream, G, p->H, p->W,
                       p->d_s, sx, ox, sy, oy, p->dRed);
    int st = hip_status(hipGetLastError(), "bg_grad_kernel");
    if (st) return st;
    hipLaunchKernelGGL(bg_grad_final, dim3(1), dim3(64), 0, p->stream, p->dRed, p->M, gb);
    return hip_status(hipGetLastError(), "bg_grad_final");
}

// ------------------------------------------- preconditioned CG ----

// Scalars of the iteration, in the plan's vector scratch after the vectors.
enum { CG_RZ = 0, CG_RR = 1 };

// r = -g / 2 (g = dL/da = 2 J^T mask (J a - I)), so r = J^T mask (I - J a)
__global__ void cg_init_kernel(const double* __restrict__ g, double* __restrict__ r, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) r[i] = -0.5 * g[i];
}

__device__ double block_dot(const double* __restrict__ u, const double* __restrict__ v, int n,
                            double* red) {
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 1024) s += u[i] * v[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    const double out = red[0];
    __syncthreads();
    return out;
}

// first direction: p = z, rz = r.z
__global__ __launch_bounds__(1024) void cg_start_kernel(const double* __restrict__ r,
                                                        const double* __restrict__ z,
                                                        double* __restrict__ pv, int n,
                                                        double* __restrict__ sc) {
    __shared__ double red[1024];
    const double rz = block_dot(r, z, n, red);
    for (int i = threadIdx.x; i < n; i += 1024) pv[i] = z[i];
    if (threadIdx.x == 0) sc[CG_RZ] = rz;
}

// q2 = 2 A p (from the adjoint of the masked loss); alpha = rz / (p.A p);
// a += alpha p; r -= alpha A p; a32 = float(a); rr = r.r
__global__ __launch_bounds__(1024) void cg_step_kernel(const double* __restrict__ pv,
                                                       const double* __restrict__ q2,
                                                       double* __restrict__ a64,
                                                       float* __restrict__ a32,
                                                       double* __restrict__ r, int n,
                                                       double* __restrict__ sc) {
    __shared__ double red[1024];
    const double pq = 0.5 * block_dot(pv, q2, n, red);
    const double alpha = (pq > 0.0 && isfinite(pq)) ? sc[CG_RZ] / pq : 0.0;
    for (int i = threadIdx.x; i < n; i += 1024) {
        const double v = a64[i] + alpha * pv[i];
        a64[i] = v;
        a32[i] = (float)v;
        r[i] -= alpha * 0.5 * q2[i];
    }
    __syncthreads();
    const double rr = block_dot(r, r, n, red);
    if (threadIdx.x == 0) sc[CG_RR] = sqrt(rr);
}

// beta = r.z / rz; p = z + beta p; rz = r.z
__global__ __launch_bounds__(1024) void cg_direction_kernel(const double* __restrict__ r,
                                                            const double* __restrict__ z,
                                                            double* __restrict__ pv, int n,
                                                            double* __restrict__ sc) {
    __shared__ double red[1024];
    const double rz_new = block_dot(r, z, n, red);
    const double rz = sc[CG_RZ];
    const double beta = (rz > 0.0 && isfinite(rz_new)) ? rz_new / rz : 0.0;
    for (int i = threadIdx.x; i < n; i += 1024) pv[i] = z[i] + beta * pv[i];
    if (threadIdx.x == 0) sc[CG_RZ] = rz_new;
}

__global__ void to_float_kernel(const double* __restrict__ v, float* __restrict__ out, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (float)v[i];
}

// g = dL/d(a, b) of L = sum_mask D^2 for the D already in `D`, into g[n]
static int loss_gradient(svconv_plan* p, const float* R, float* D, const unsigned char* mask,
                         double* g) {
    int st = launch_loss_grad(p, D, mask, p->dGrad, nullptr);
    if (!st) st = launch_adjoint_a(p, R, p->dGrad, g);
    if (!st && p->bg) st = launch_bg_grad(p, p->dGrad, g + (size_t)p->N * p->M);
    return st;
}

}  // namespace svc

using namespace svc;

extern "C" {

int svconv_stamp_mask(svconv_plan* p, const float* R, double sky, double threshold, double frac,
                      int r_iso, int margin, int stamp_half, unsigned char* mask, int* n_centres) {
    if (!p || !R || !mask) return fail(SVCONV_EINVAL, "NULL argument");
    if (!std::isfinite(sky) || !std::isfinite(threshold)) return fail(SVCONV_EINVAL, "sky and threshold must be finite");
    if (!(frac > 0.0) || !std::isfinite(frac)) return fail(SVCONV_EINVAL, "frac must be positive");
    if (r_iso < 1 || r_iso > 64) return fail(SVCONV_EINVAL, "r_iso must be in [1, 64]");
    if (stamp_half < 0 || stamp_half > 64) return fail(SVCONV_EINVAL, "stamp_half must be in [0, 64]");
    if (margin < 0) return fail(SVCONV_EINVAL, "margin < 0");
    const size_t n = (size_t)p->H * p->W;
    unsigned char* flags = reinterpret_cast<unsigned char*>(p->dGrad);   // n bytes
    unsigned char* rows = flags + n;                                     // n bytes (dGrad holds 4 n)
    hipLaunchKernelGGL(centre_kernel, dim3(2048), dim3(256), 0, p->stream, R, p->H, p->W, sky,
                       threshold, frac, r_iso, margin, flags);
    int st = hip_status(hipGetLastError(), "centre_kernel");
    if (st) return st;
    hipLaunchKernelGGL(dilate_rows_kernel, dim3(2048), dim3(256), 0, p->stream, flags, p->H, p->W,
                       stamp_half, rows);
    st = hip_status(hipGetLastError(), "dilate_rows_kernel");
    if (st) return st;
    hipLaunchKernelGGL(dilate_cols_kernel, dim3(2048), dim3(256), 0, p->stream, rows, p->H, p->W,
                       stamp_half, mask);
    st = hip_status(hipGetLastError(), "dilate_cols_kernel");
    if (st || !n_centres) return st;
    int* part = reinterpret_cast<int*>(p->dRed);
    hipLaunchKernelGGL(count_kernel, dim3(COUNT_BLOCKS), dim3(256), 0, p->stream, flags, n, part);
    st = hip_status(hipGetLastError(), "count_kernel");
    if (st) return st;
    hipLaunchKernelGGL(count_total_kernel, dim3(1), dim3(64), 0, p->stream, part);
    st = hip_status(hipGetLastError(), "count_total_kernel");
    if (st) return st;
    int total = 0;
    st = hip_status(hipMemcpyAsync(&total, part + COUNT_BLOCKS, sizeof(int), hipMemcpyDeviceToHost,
                                   p->stream), "copy count");
    if (!st) st = hip_status(hipStreamSynchronize(p->stream), "hipStreamSynchronize");
    if (!st) *n_centres = total;
    return st;
}

int svconv_plan_set_background(svconv_plan* p, int enable) {
    if (!p) return fail(SVCONV_EINVAL, "plan is NULL");
    if (enable != 0 && enable != 1) return fail(SVCONV_EINVAL, "enable must be 0 or 1");
    if (enable && (p->N + 1 > kMaxFilters || (p->N + 1) * p->M > kMaxCoefficients))
        return fail(SVCONV_EUNSUPPORTED, "background needs N + 1 <= 64 and (N + 1) M <= 1024");
    p->bg = enable;
    return SVCONV_OK;
}

int svconv_add_background(svconv_plan* p, const float* b, float* D) {
    if (!p || !b || !D) return fail(SVCONV_EINVAL, "NULL argument");
    return launch_add_background(p, b, D);
}

int svconv_pcg_fit(svconv_plan* p, const float* R, const float* I, const unsigned char* mask,
                   const double* L, int iters, double* a64, float* a32, float* D,
                   double* host_residuals) {
    if (!p || !R || !I || !L || !a64 || !a32 || !D) return fail(SVCONV_EINVAL, "NULL argument");
    if ((const void*)D == (const void*)R || (const void*)D == (const void*)I)
        return fail(SVCONV_EINVAL, "D aliases R or I");
    if (iters < 0 || iters > 10000) return fail(SVCONV_EINVAL, "iters must be in [0, 10000]");
    const int NK = p->N * p->M;
    const int n = NK + p->bg * p->M;
    double* r = p->dVec;
    double* z = r + n;
    double* pv = z + n;
    double* q = pv + n;
    double* sc = q + n;                                    // 8 scalars
    float* p32 = reinterpret_cast<float*>(sc + 8);         // n floats
    const dim3 vec_grid((n + 255) / 256);
    // r = J^T mask (I - J a), z = M^-1 r, p = z
    hipLaunchKernelGGL(to_float_kernel, vec_grid, dim3(256), 0, p->stream, a64, a32, n);
    int st = hip_status(hipGetLastError(), "to_float_kernel");
    if (!st) st = run_forward(p, R, I, a32, D);
    if (!st && p->bg) st = launch_add_background(p, a32 + NK, D);
    if (!st) st = loss_gradient(p, R, D, mask, q);
    if (!st) {
        hipLaunchKernelGGL(cg_init_kernel, dim3(1), dim3(1024), 0, p->stream, q, r, n);
        st = hip_status(hipGetLastError(), "cg_init_kernel");
    }
    if (!st) st = launch_cholesky_solve(p, L, r, z, n);
    if (!st) {
        hipLaunchKernelGGL(cg_start_kernel, dim3(1), dim3(1024), 0, p->stream, r, z, pv, n, sc);
        st = hip_status(hipGetLastError(), "cg_start_kernel");
    }
    for (int it = 0; it < iters && !st; ++it) {
        // q = 2 J^T mask J p: forward of the direction without I, then the
        // adjoint of the masked loss at that image
        hipLaunchKernelGGL(to_float_kernel, vec_grid, dim3(256), 0, p->stream, pv, p32, n);
        st = hip_status(hipGetLastError(), "to_float_kernel");
        if (!st) st = run_forward(p, R, nullptr, p32, D);
        if (!st && p->bg) st = launch_add_background(p, p32 + NK, D);
        if (!st) st = loss_gradient(p, R, D, mask, q);
        if (!st) {
            hipLaunchKernelGGL(cg_step_kernel, dim3(1), dim3(1024), 0, p->stream, pv, q, a64, a32,
                               r, n, sc);
            st = hip_status(hipGetLastError(), "cg_step_kernel");
        }
        if (!st && host_residuals)
            st = hip_status(hipMemcpyAsync(host_residuals + it, sc + CG_RR, sizeof(double),
                                           hipMemcpyDeviceToHost, p->stream), "copy residual");
        if (!st) st = launch_cholesky_solve(p, L, r, z, n);
        if (!st) {
            hipLaunchKernelGGL(cg_direction_kernel, dim3(1), dim3(1024), 0, p->stream, r, z, pv, n,
                               sc);
            st = hip_status(hipGetLastError(), "cg_direction_kernel");
        }
    }
    // D at the final coefficients
    if (!st) st = run_forward(p, R, I, a32, D);
    if (!st && p->bg) st = launch_add_background(p, a32 + NK, D);
    if (!st && host_residuals) st = hip_status(hipStreamSynchronize(p->stream), "hipStreamSynchronize");
    return st;
}

}  // extern "C"
