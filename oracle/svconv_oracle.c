/*
 * Plain FP64 CPU oracle for spatially-varying-kernel image convolution and
 * subtraction (Hartung, Shukla, Miller & Pennypacker, "GPU acceleration of
 * image convolution using spatially-varying kernel").
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg call this code.  It is written to be read
 * against the paper, not to be fast: every pixel builds its own kernel and
 * convolves directly, as the paper's Sec. 3 says the method does ("the best
 * available kernel at every pixel").  It shares no code, header or table
 * with the GPU library.
 *
 * Conventions (readings where the paper is silent; each is listed with its
 * reason in the design notes of the repository):
 *   - images are row-major [H][W], x = column, y = row;
 *   - the basis functions are Gaussians times monomials u^i v^j (u along x,
 *     v along y), each scaled to unit L1 norm; sigma = 0 means a Kronecker
 *     delta at (0,0);
 *   - coordinates are normalised over the full frame,
 *     xh = 2 (x + x0) / (Wf - 1) - 1, yh likewise (0 for a 1-pixel axis);
 *   - spatial terms are xh^i yh^j listed by total degree, then descending i;
 *   - (R (x) K)(x,y) = sum_{u,v} K(x,y)[u,v] R(x-u, y-v): true convolution,
 *     with the kernel taken at the output pixel and R = 0 outside the array.
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC svconv_oracle.c -o liboracle.so -lm
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)
#define ORC_ENOTSPD (-5)

/* x^i with 0^0 = 1, by repeated multiplication. */
static double ipow(double x, int i)
{
    double r = 1.0;
    for (int t = 0; t < i; ++t) r *= x;
    return r;
}

int orc_n_basis(int n_gauss, const int* degrees)
{
    int n = 0;
    for (int g = 0; g < n_gauss; ++g) n += (degrees[g] + 1) * (degrees[g] + 2) / 2;
    return n;
}

int orc_n_spatial(int d_s) { return (d_s + 1) * (d_s + 2) / 2; }

/* Spatial degrees above this are rejected (fixed-size term buffers below). */
#define ORC_MAX_SPATIAL_DEGREE 9

/*
 * Basis functions B_n (Sec. 2, Eq. 2: the kernel is a weighted sum of basis
 * functions; the Gaussian basis of Alard & Lupton, cited in Sec. 2).
 * out[n][(v+h)*k + (u+h)], k = 2h+1.
 */
int orc_basis(int h, int n_gauss, const double* sigmas, const int* degrees, double* out)
{
    if (h < 0 || n_gauss <= 0) return ORC_EINVAL;
    const int k = 2 * h + 1;
    int n = 0;
    for (int g = 0; g < n_gauss; ++g) {
        const double s = sigmas[g];
        const int d = degrees[g];
        if (s < 0.0 || d < 0 || (s == 0.0 && d != 0)) return ORC_EINVAL;
        for (int t = 0; t <= d; ++t) {
            for (int i = t; i >= 0; --i) {
                const int j = t - i;
                double* B = out + (size_t)n * k * k;
                double l1 = 0.0;
                for (int v = -h; v <= h; ++v) {
                    for (int u = -h; u <= h; ++u) {
                        double val;
                        if (s == 0.0)
                            val = (u == 0 && v == 0) ? 1.0 : 0.0;
                        else
                            val = exp(-(double)(u * u + v * v) / (2.0 * s * s)) * ipow(u, i) * ipow(v, j);
                        B[(v + h) * k + (u + h)] = val;
                        l1 += fabs(val);
                    }
                }
                if (l1 > 0.0)
                    for (int q = 0; q < k * k; ++q) B[q] /= l1;
                ++n;
            }
        }
    }
    return n;
}

/*
 * Dirac delta basis (Sec. 2: one basis function per kernel pixel): basis
 * n = (v+h) k + (u+h) is 1 at (u, v) and 0 elsewhere.  out[n][k][k].
 */
int orc_basis_dfb(int h, double* out)
{
    if (h < 0) return ORC_EINVAL;
    const int k = 2 * h + 1;
    const int N = k * k;
    for (int n = 0; n < N; ++n)
        for (int q = 0; q < N; ++q) out[(size_t)n * N + q] = (q == n) ? 1.0 : 0.0;
    return N;
}

/* Normalised full-frame coordinate of an array index (frame offset off). */
static double norm_coord(int idx, int off, int frame)
{
    if (frame <= 1) return 0.0;
    return 2.0 * (double)(idx + off) / (double)(frame - 1) - 1.0;
}

/* Spatial terms P_m (Eq. 3, generalised to degree d_s): xh^i yh^j. */
void orc_spatial_terms(double xh, double yh, int d_s, double* P)
{
    int m = 0;
    for (int t = 0; t <= d_s; ++t)
        for (int i = t; i >= 0; --i) P[m++] = ipow(xh, i) * ipow(yh, t - i);
}

/* Per-pixel coefficients c_n = sum_m a[n][m] P_m (the polynomial scaling of
 * each basis in Eq. 2, Eq. 3). */
static void coeffs_at(int N, int M, const double* a, const double* P, double* c)
{
    for (int n = 0; n < N; ++n) {
        double s = 0.0;
        for (int m = 0; m < M; ++m) s += a[n * M + m] * P[m];
        c[n] = s;
    }
}

/* The kernel at one pixel, K[(v+h)*k+(u+h)] = sum_n c_n B_n (Eq. 2). */
static void kernel_from_coeffs(int k, int N, const double* basis, const double* c, double* K)
{
    for (int q = 0; q < k * k; ++q) {
        double s = 0.0;
        for (int n = 0; n < N; ++n) s += c[n] * basis[(size_t)n * k * k + q];
        K[q] = s;
    }
}

/* K(x,y) at array pixel (x, y), exported for the tests' brute force. */
int orc_kernel_at(int x, int y, int h, int N, const double* basis, int d_s, const double* a,
                  int x0, int y0, int Wf, int Hf, double* K)
{
    const int M = orc_n_spatial(d_s);
    double* P = (double*)malloc(sizeof(double) * M);
    double* c = (double*)malloc(sizeof(double) * N);
    if (!P || !c) { free(P); free(c); return ORC_ENOMEM; }
    orc_spatial_terms(norm_coord(x, x0, Wf), norm_coord(y, y0, Hf), d_s, P);
    coeffs_at(N, M, a, P, c);
    kernel_from_coeffs(2 * h + 1, N, basis, c, K);
    free(P); free(c);
    return ORC_OK;
}

/* C(x,y) = sum_{u,v} K(x,y)[u,v] R(x-u, y-v) with R = 0 outside (Eq. 1, 2). */
static double convolve_pixel(int H, int W, const double* R, int h, const double* K, int x, int y)
{
    const int k = 2 * h + 1;
    double acc = 0.0;
    for (int v = -h; v <= h; ++v) {
        const int ys = y - v;
        if (ys < 0 || ys >= H) continue;
        for (int u = -h; u <= h; ++u) {
            const int xs = x - u;
            if (xs < 0 || xs >= W) continue;
            acc += K[(v + h) * k + (u + h)] * R[(size_t)ys * W + xs];
        }
    }
    return acc;
}

static void set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

/* Full convolution R (x) K(x,y) (Eq. 1 without the subtraction). */
int orc_convolve(int H, int W, const double* R, int h, int N, const double* basis, int d_s,
                 const double* a, int x0, int y0, int Wf, int Hf, double* C, int nthreads)
{
    if (H <= 0 || W <= 0 || h < 0 || N <= 0 || d_s < 0 || d_s > ORC_MAX_SPATIAL_DEGREE) return ORC_EINVAL;
    const int k = 2 * h + 1;
    const int M = orc_n_spatial(d_s);
    int err = 0;
    set_threads(nthreads);
#pragma omp parallel
    {
        double* P = (double*)malloc(sizeof(double) * M);
        double* c = (double*)malloc(sizeof(double) * N);
        double* K = (double*)malloc(sizeof(double) * k * k);
        const int ok = (P && c && K);
        if (!ok) {
#pragma omp atomic write
            err = 1;
        }
        /* every thread meets the work-sharing loop; one without buffers skips its rows */
#pragma omp for schedule(static)
        for (int y = 0; y < H; ++y) {
            if (!ok) continue;
            for (int x = 0; x < W; ++x) {
                orc_spatial_terms(norm_coord(x, x0, Wf), norm_coord(y, y0, Hf), d_s, P);
                coeffs_at(N, M, a, P, c);
                kernel_from_coeffs(k, N, basis, c, K);
                C[(size_t)y * W + x] = convolve_pixel(H, W, R, h, K, x, y);
            }
        }
        free(P); free(c); free(K);
    }
    return err ? ORC_ENOMEM : ORC_OK;
}

/* The same convolution at a list of array pixels (xs[i], ys[i]). */
int orc_convolve_at(int H, int W, const double* R, int h, int N, const double* basis, int d_s,
                    const double* a, int x0, int y0, int Wf, int Hf, int npts, const int* xs,
                    const int* ys, double* out, int nthreads)
{
    if (H <= 0 || W <= 0 || h < 0 || N <= 0 || d_s < 0 || d_s > ORC_MAX_SPATIAL_DEGREE || npts < 0) return ORC_EINVAL;
    const int k = 2 * h + 1;
    const int M = orc_n_spatial(d_s);
    for (int i = 0; i < npts; ++i)
        if (xs[i] < 0 || xs[i] >= W || ys[i] < 0 || ys[i] >= H) return ORC_EINVAL;
    int err = 0;
    set_threads(nthreads);
#pragma omp parallel
    {
        double* P = (double*)malloc(sizeof(double) * M);
        double* c = (double*)malloc(sizeof(double) * N);
        double* K = (double*)malloc(sizeof(double) * k * k);
        const int ok = (P && c && K);
        if (!ok) {
#pragma omp atomic write
            err = 1;
        }
#pragma omp for schedule(dynamic, 16)
        for (int i = 0; i < npts; ++i) {
            if (!ok) continue;
            orc_spatial_terms(norm_coord(xs[i], x0, Wf), norm_coord(ys[i], y0, Hf), d_s, P);
            coeffs_at(N, M, a, P, c);
            kernel_from_coeffs(k, N, basis, c, K);
            out[i] = convolve_pixel(H, W, R, h, K, xs[i], ys[i]);
        }
        free(P); free(c); free(K);
    }
    return err ? ORC_ENOMEM : ORC_OK;
}

/* T_n(x,y) = sum_{u,v} B_n[u,v] R(x-u, y-v): one basis convolved with R. */
static double basis_response(int H, int W, const double* R, int h, const double* Bn, int x, int y)
{
    return convolve_pixel(H, W, R, h, Bn, x, y);
}

/*
 * Gradient of L with respect to the coefficients, given G = dL/dD:
 * dL/da[n][m] = sum_{x,y} G(x,y) P_m(x,y) T_n(x,y), because D is linear in a
 * through Eq. 2 and Eq. 3.
 */
int orc_grad_a(int H, int W, const double* R, int h, int N, const double* basis, int d_s,
               int x0, int y0, int Wf, int Hf, const double* G, double* ga, int nthreads)
{
    if (H <= 0 || W <= 0 || h < 0 || N <= 0 || d_s < 0 || d_s > ORC_MAX_SPATIAL_DEGREE) return ORC_EINVAL;
    const int k = 2 * h + 1;
    const int M = orc_n_spatial(d_s);
    int nt = 1;
    set_threads(nthreads);
#ifdef _OPENMP
#pragma omp parallel
    {
#pragma omp single
        nt = omp_get_num_threads();
    }
#endif
    double* part = (double*)calloc((size_t)nt * N * M, sizeof(double));
    if (!part) return ORC_ENOMEM;
#pragma omp parallel num_threads(nt)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double* acc = part + (size_t)tid * N * M;
        double P[64];
#pragma omp for schedule(static)
        for (int y = 0; y < H; ++y) {
            for (int x = 0; x < W; ++x) {
                const double g = G[(size_t)y * W + x];
                if (g == 0.0) continue;
                orc_spatial_terms(norm_coord(x, x0, Wf), norm_coord(y, y0, Hf), d_s, P);
                for (int n = 0; n < N; ++n) {
                    const double T = basis_response(H, W, R, h, basis + (size_t)n * k * k, x, y);
                    for (int m = 0; m < M; ++m) acc[n * M + m] += g * P[m] * T;
                }
            }
        }
    }
    for (int q = 0; q < N * M; ++q) {
        double s = 0.0;
        for (int t = 0; t < nt; ++t) s += part[(size_t)t * N * M + q];
        ga[q] = s;
    }
    free(part);
    return ORC_OK;
}

/*
 * Gradient of L with respect to the reference image, given G = dL/dD:
 * C(p) depends on R(q) through K(p)[p-q], so
 * dL/dR(q) = sum_{u,v} G(q+(u,v)) K(q+(u,v))[u,v] over in-array pixels.
 */
int orc_grad_R(int H, int W, int h, int N, const double* basis, int d_s, const double* a,
               int x0, int y0, int Wf, int Hf, const double* G, double* gR, int nthreads)
{
    if (H <= 0 || W <= 0 || h < 0 || N <= 0 || d_s < 0 || d_s > ORC_MAX_SPATIAL_DEGREE) return ORC_EINVAL;
    const int k = 2 * h + 1;
    const int M = orc_n_spatial(d_s);
    /* per-pixel coefficients c_n(p), kept for all pixels */
    double* c = (double*)malloc(sizeof(double) * (size_t)H * W * N);
    if (!c) return ORC_ENOMEM;
    set_threads(nthreads);
#pragma omp parallel
    {
        double P[64];
#pragma omp for schedule(static)
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x) {
                orc_spatial_terms(norm_coord(x, x0, Wf), norm_coord(y, y0, Hf), d_s, P);
                coeffs_at(N, M, a, P, c + ((size_t)y * W + x) * N);
            }
#pragma omp for schedule(static)
        for (int y = 0; y < H; ++y) {
            for (int x = 0; x < W; ++x) {
                double acc = 0.0;
                for (int v = -h; v <= h; ++v) {
                    const int py = y + v;
                    if (py < 0 || py >= H) continue;
                    for (int u = -h; u <= h; ++u) {
                        const int px = x + u;
                        if (px < 0 || px >= W) continue;
                        const double* cp = c + ((size_t)py * W + px) * N;
                        double Kuv = 0.0;
                        for (int n = 0; n < N; ++n) Kuv += cp[n] * basis[(size_t)n * k * k + (v + h) * k + (u + h)];
                        acc += G[(size_t)py * W + px] * Kuv;
                    }
                }
                gR[(size_t)y * W + x] = acc;
            }
        }
    }
    free(c);
    return ORC_OK;
}

/*
 * Normal equations of the least-squares fit of the coefficients (OIS, Sec. 2):
 * with Phi[p][(n,m)] = P_m(p) T_n(p), JtJ = Phi^T Phi and rhs = Phi^T I,
 * summed over pixels with mask[p] != 0 (mask NULL: the interior, at least h
 * pixels from every edge).  Index (n,m) -> n*M + m.  Small problems only.
 */
int orc_normal_equations(int H, int W, const double* R, const double* I, int h, int N,
                         const double* basis, int d_s, int x0, int y0, int Wf, int Hf,
                         const unsigned char* mask, double* JtJ, double* rhs)
{
    if (H <= 0 || W <= 0 || h < 0 || N <= 0 || d_s < 0 || d_s > ORC_MAX_SPATIAL_DEGREE) return ORC_EINVAL;
    const int k = 2 * h + 1;
    const int M = orc_n_spatial(d_s);
    const int NM = N * M;
    double* phi = (double*)malloc(sizeof(double) * NM);
    double* T = (double*)malloc(sizeof(double) * N);
    if (!phi || !T) { free(phi); free(T); return ORC_ENOMEM; }
    memset(JtJ, 0, sizeof(double) * (size_t)NM * NM);
    if (rhs) memset(rhs, 0, sizeof(double) * NM);
    double P[64];
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            int use;
            if (mask) use = mask[(size_t)y * W + x] != 0;
            else use = (x >= h && x <= W - 1 - h && y >= h && y <= H - 1 - h);
            if (!use) continue;
            orc_spatial_terms(norm_coord(x, x0, Wf), norm_coord(y, y0, Hf), d_s, P);
            for (int n = 0; n < N; ++n) T[n] = basis_response(H, W, R, h, basis + (size_t)n * k * k, x, y);
            for (int n = 0; n < N; ++n)
                for (int m = 0; m < M; ++m) phi[n * M + m] = P[m] * T[n];
            for (int i = 0; i < NM; ++i)
                for (int j = 0; j < NM; ++j) JtJ[(size_t)i * NM + j] += phi[i] * phi[j];
            if (rhs && I)
                for (int i = 0; i < NM; ++i) rhs[i] += phi[i] * I[(size_t)y * W + x];
        }
    }
    free(phi); free(T);
    return ORC_OK;
}

/* Solve A x = b for symmetric positive definite A (n x n, row-major) by the
 * Cholesky factorisation A = L L^T, then two triangular solves. */
int orc_cholesky_solve(int n, const double* A, const double* b, double* x)
{
    if (n <= 0) return ORC_EINVAL;
    double* L = (double*)calloc((size_t)n * n, sizeof(double));
    if (!L) return ORC_ENOMEM;
    for (int j = 0; j < n; ++j) {
        double d = A[(size_t)j * n + j];
        for (int p = 0; p < j; ++p) d -= L[(size_t)j * n + p] * L[(size_t)j * n + p];
        if (!(d > 0.0)) { free(L); return ORC_ENOTSPD; }
        const double ljj = sqrt(d);
        L[(size_t)j * n + j] = ljj;
        for (int i = j + 1; i < n; ++i) {
            double s = A[(size_t)i * n + j];
            for (int p = 0; p < j; ++p) s -= L[(size_t)i * n + p] * L[(size_t)j * n + p];
            L[(size_t)i * n + j] = s / ljj;
        }
    }
    /* L z = b */
    for (int i = 0; i < n; ++i) {
        double s = b[i];
        for (int p = 0; p < i; ++p) s -= L[(size_t)i * n + p] * x[p];
        x[i] = s / L[(size_t)i * n + i];
    }
    /* L^T x = z */
    for (int i = n - 1; i >= 0; --i) {
        double s = x[i];
        for (int p = i + 1; p < n; ++p) s -= L[(size_t)p * n + i] * x[p];
        x[i] = s / L[(size_t)i * n + i];
    }
    free(L);
    return ORC_OK;
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
