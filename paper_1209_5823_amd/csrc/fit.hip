// Least-squares fit of the coefficients (Optimal Image Subtraction, Sec. 2):
// loss and its gradient in D, the float64 normal matrix, an in-place
// Cholesky factorisation, the two triangular solves and the Gauss-Newton
// update.  Everything here is float64 except the basis responses, which come
// from the float32 matrix-core contraction.
//
// Normal matrix.  With Phi[p][(n,m)] = P_m(p) T_n(p),
//   JtJ[(n,m)][(n',m')] = sum_p mask(p) T_n(p) T_n'(p) P_m(p) P_m'(p),
// and P_m P_m' is itself one monomial xh^(i+i') yh^(j+j') of degree at most
// 2 d_s.  So JtJ is assembled from
//   S[mu][n][n'] = sum_p mask(p) Q_mu(p) T_n(p) T_n'(p)
// over the (d_s + 1)(2 d_s + 1) monomials Q_mu of degree <= 2 d_s, which needs
// N^2 per monomial instead of (N M)^2 products per pixel.  Within one image
// row yh is constant, so with Q_mu = xh^a yh^b the Gram sums of a row segment
// are taken for the 2 d_s + 1 powers of xh only,
//   G_a[n][n'] = sum_{x in segment} mask xh^a T_n T_n',
// and S[(a, b)] = sum_segments yh^b G_a is formed by the reduction: 2 d_s + 1
// instead of (d_s + 1)(2 d_s + 1) weighted products per pixel.  The T_n of a
// band of rows are produced by the forward contraction (written out instead
// of being contracted with c_n), then G is accumulated on the float64 matrix
// cores (v_mfma_f64_16x16x4_f64).
#include <cmath>

#include "internal.hpp"

namespace svc {

typedef double d4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------ loss ----

__device__ __forceinline__ bool in_mask(const unsigned char* mask, int H, int W, int h, int x, int y) {
    if (mask) return mask[(size_t)y * W + x] != 0;
    return x >= h && x <= W - 1 - h && y >= h && y <= H - 1 - h;
}

constexpr int LOSS_BLOCKS = 1024;

__global__ void loss_grad_kernel(const float* __restrict__ D, const unsigned char* __restrict__ mask,
                                 int H, int W, int h, float* __restrict__ gD,
                                 double* __restrict__ part) {
    double s = 0.0;
    const size_t n = (size_t)H * W;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const int y = (int)(i / W), x = (int)(i % W);
        const float d = D[i];
        const bool m = in_mask(mask, H, W, h, x, y);
        gD[i] = m ? 2.f * d : 0.f;
        if (m) s += (double)d * d;
    }
    __shared__ double red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void sum_kernel(const double* __restrict__ part, int n, double* __restrict__ out) {
    __shared__ double red[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

int launch_loss_grad(svconv_plan* p, const float* D, const unsigned char* mask, float* gD,
                     double* loss) {
    hipLaunchKernelGGL(loss_grad_kernel, dim3(LOSS_BLOCKS), dim3(256), 0, p->stream, D, mask, p->H,
                       p->W, p->h, gD, p->dRed);
    int st = hip_status(hipGetLastError(), "loss_grad_kernel");
    if (st || !loss) return st;
    hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(256), 0, p->stream, p->dRed, LOSS_BLOCKS, loss);
    return hip_status(hipGetLastError(), "sum_kernel");
}

// --------------------------------------------------- normal matrix ----

constexpr int NM_PIX_CHUNK = 4096;    // pixels per workgroup and band
constexpr size_t NM_BAND_BYTES = (size_t)512 << 20;

__device__ __forceinline__ double ipow_f(double x, int e) {
    double r = 1.0;
    for (int t = 0; t < e; ++t) r *= x;
    return r;
}

// G_part[seg][a][n][n'] for 64 x 64 (n, n') and one power a of xh per
// workgroup; a segment is up to NM_PIX_CHUNK pixels of one row of the band.
// The 16 x 16 blocks with row block <= column block are formed (the waves
// share them out); blocks whose rows or columns are all padding are skipped.
// A operand: T_n(p_k); B operand: T_n'(p_k) xh^a mask.
constexpr int GRAM_WAVES = 5;   // two of the 10 block pairs per wave

__global__ __launch_bounds__(64 * GRAM_WAVES) void gram_kernel(const float* __restrict__ T, int N, int band_px,
                                                   int y_begin, int W, int H, int h, int cpr,
                                                   const unsigned char* __restrict__ mask,
                                                   double sx, double ox, int n_a,
                                                   double* __restrict__ part) {
    const int ea = blockIdx.x;
    const int seg = blockIdx.y;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int kq = lane >> 4, j = lane & 15;
    const int row = seg / cpr, x_begin = (seg - row * cpr) * NM_PIX_CHUNK;
    const int x_end = min(W, x_begin + NM_PIX_CHUNK);
    const int y = y_begin + row;

    // G is symmetric: only the 10 blocks (rb, cb) with rb <= cb of the 4 x 4
    // block grid are formed, two of them by each of the 5 waves (equal work
    // on every SIMD)
    constexpr int PAIRS[10][2] = {{0, 0}, {0, 1}, {0, 2}, {0, 3}, {1, 1},
                                  {1, 2}, {1, 3}, {2, 2}, {2, 3}, {3, 3}};
    constexpr int PQ = 2;
    const int p_begin = PQ * w;
    d4 acc[PQ];
#pragma unroll
    for (int q = 0; q < PQ; ++q) acc[q] = d4{0.0, 0.0, 0.0, 0.0};
    // 16 pixels per step: lane group kq takes pixels x0 + 4 kq .. x0 + 4 kq + 3
    // (the k slot of instruction s is pixel x0 + 4 kq + s in both operands),
    // so each lane reads 4 consecutive floats of a filter row
    const bool vec = (W & 3) == 0;
    // pixel weights xh^ea (0 outside the mask) of the segment, formed once
    // per workgroup (x^ea from the binary digits of ea <= 12)
    __shared__ double wsh[NM_PIX_CHUNK];
    for (int i = threadIdx.x; i < x_end - x_begin; i += 64 * GRAM_WAVES) {
        const int x = x_begin + i;
        const double xh = sx * x + ox, x2 = xh * xh, x4 = x2 * x2, x8 = x4 * x4;
        wsh[i] = in_mask(mask, H, W, h, x, y) ? ((ea & 1) ? xh : 1.0) * ((ea & 2) ? x2 : 1.0) *
                                                     ((ea & 4) ? x4 : 1.0) * ((ea & 8) ? x8 : 1.0)
                                               : 0.0;
    }
    __syncthreads();
    // the lane's block rows of its two block pairs; every operand load
    // below is unconditional, from a clamped row
    const float* tb = T + (size_t)row * W + 4 * kq;
    size_t offa[PQ], offb[PQ];
    bool use[PQ], ina[PQ], inb[PQ];
#pragma unroll
    for (int q = 0; q < PQ; ++q) {
        const int pi = p_begin + q;
        const int rb = PAIRS[pi][0], cb = PAIRS[pi][1];
        use[q] = 16 * rb < N && 16 * cb < N;   // uniform
        ina[q] = 16 * rb + j < N;
        inb[q] = 16 * cb + j < N;
        offa[q] = (size_t)min(16 * rb + j, N - 1) * band_px;
        offb[q] = (size_t)min(16 * cb + j, N - 1) * band_px;
    }
    int x0 = x_begin;
    if (vec) {
        // the steps whose 16 pixels are all inside the segment, two per turn:
        // the operands of one step are requested (into a register set of
        // their own) before the products of the step before it
        const int x_full = x_begin + (x_end - x_begin) / 16 * 16;
        auto load_step = [&](int xs, float4 (&o)[PQ][2]) {
#pragma unroll
            for (int q = 0; q < PQ; ++q) {
                o[q][0] = *reinterpret_cast<const float4*>(tb + offa[q] + xs);
                o[q][1] = *reinterpret_cast<const float4*>(tb + offb[q] + xs);
            }
        };
        auto run_step = [&](int xs, const float4 (&o)[PQ][2]) {
            const double* wp = wsh + (xs - x_begin + 4 * kq);
            double wq[4];
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) wq[s4] = wp[s4];
#pragma unroll
            for (int q = 0; q < PQ; ++q) {
                if (use[q]) {
                    const float av[4] = {o[q][0].x, o[q][0].y, o[q][0].z, o[q][0].w};
                    const float bv[4] = {o[q][1].x, o[q][1].y, o[q][1].z, o[q][1].w};
#pragma unroll
                    for (int s4 = 0; s4 < 4; ++s4)
                        acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                            ina[q] ? (double)av[s4] : 0.0, inb[q] ? (double)bv[s4] * wq[s4] : 0.0,
                            acc[q], 0, 0, 0);
                }
            }
        };
        float4 oA[PQ][2], oB[PQ][2];
        if (x0 < x_full) load_step(x0, oA);
        for (; x0 + 32 <= x_full; x0 += 32) {
            load_step(x0 + 16, oB);
            run_step(x0, oA);
            load_step(x0 + 32 < x_full ? x0 + 32 : x0 + 16, oA);   // past the end: unused
            run_step(x0 + 16, oB);
        }
        if (x0 < x_full) {
            run_step(x0, oA);
            x0 += 16;
        }
    }
    // the remaining pixels (all of them when W is not a multiple of 4)
    for (; x0 < x_end; x0 += 16) {
        const int xb = x0 + 4 * kq;
        const size_t pb = (size_t)row * W + xb;
        double wq[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) wq[s] = (xb + s < x_end) ? wsh[xb + s - x_begin] : 0.0;
        auto load4 = [&](int nrow, float* v) {
            v[0] = v[1] = v[2] = v[3] = 0.f;
            if (nrow < N) {
                const float* src = T + (size_t)nrow * band_px + pb;
#pragma unroll
                for (int s = 0; s < 4; ++s) v[s] = (xb + s < x_end) ? src[s] : 0.f;
            }
        };
#pragma unroll
        for (int q = 0; q < PQ; ++q) {
            {
                const int rb = PAIRS[p_begin + q][0], cb = PAIRS[p_begin + q][1];
                if (16 * rb < N && 16 * cb < N) {   // uniform
                    float av[4], bv[4];
                    load4(16 * rb + j, av);
                    load4(16 * cb + j, bv);
#pragma unroll
                    for (int s = 0; s < 4; ++s)
                        acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)av[s], (double)bv[s] * wq[s],
                                                                       acc[q], 0, 0, 0);
                }
            }
        }
    }
    // the float64 16x16x4 instruction stores row 4 e + kq of the 16 x 16
    // block in register e of lane (kq, j) (groups of one row, unlike the
    // float32 form's groups of four): lane (kq, j) holds
    // G[n = 16 rb + 4 e + kq][n' = 16 cb + j]
    double* dst = part + ((size_t)seg * n_a + ea) * 64 * 64;
#pragma unroll
    for (int q = 0; q < PQ; ++q) {
        const int rb = PAIRS[p_begin + q][0], cb = PAIRS[p_begin + q][1];
#pragma unroll
        for (int e = 0; e < 4; ++e) dst[(16 * rb + 4 * e + kq) * 64 + 16 * cb + j] = acc[q][e];
    }
}

// S[(a, b)][.][.] += sum over segments (fixed order) of yh(segment row)^b G_a
__global__ void gram_reduce(const double* __restrict__ part, int n_seg, int cpr, int n_a,
                            int y_begin, double sy, double oy, double* __restrict__ S) {
    // thread (a, e): entry e of the partial sums of x power a, read once and
    // added into S[mu(a, b)] for every y power b <= 2 d - a (n_a = 2 d + 1);
    // yh^b by repeated products, the same sums as one power at a time
    constexpr int NB_MAX = 2 * kMaxSpatialDegree + 1;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const int ea = blockIdx.y;
    if (e >= 4096) return;
    if (((e >> 6) >> 4) > ((e & 63) >> 4)) return;   // lower blocks are not formed (S symmetric)
    const int n_eb = n_a - ea;                        // uniform
    double acc[NB_MAX];
#pragma unroll
    for (int eb = 0; eb < NB_MAX; ++eb) acc[eb] = 0.0;
#pragma unroll 4
    for (int c = 0; c < n_seg; ++c) {
        const double v = part[((size_t)c * n_a + ea) * 4096 + e];
        const double yh = sy * (y_begin + c / cpr) + oy;
        double pw = 1.0;
#pragma unroll
        for (int eb = 0; eb < NB_MAX; ++eb) {
            if (eb < n_eb) acc[eb] += pw * v;
            pw *= yh;
        }
    }
#pragma unroll
    for (int eb = 0; eb < NB_MAX; ++eb) {
        if (eb < n_eb) {
            const int tt = ea + eb;
            S[(size_t)(tt * (tt + 1) / 2 + eb) * 4096 + e] += acc[eb];
        }
    }
}

__global__ void zero_kernel(double* __restrict__ v, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        v[i] = 0.0;
}

// JtJ[(n,m)][(n',m')] = S[mu(i_m + i_m', j_m + j_m')][n][n']
__global__ void assemble_jtj(const double* __restrict__ S, int N, int M, double* __restrict__ JtJ) {
    const int NM = N * M;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= NM * NM) return;
    const int r = idx / NM, c = idx % NM;
    const int n = r / M, m = r % M, n2 = c / M, m2 = c % M;
    auto expo = [](int q, int& i, int& jj) {
        int t = 0;
        while ((t + 1) * (t + 2) / 2 <= q) ++t;
        jj = q - t * (t + 1) / 2;
        i = t - jj;
    };
    int i1, j1, i2, j2;
    expo(m, i1, j1);
    expo(m2, i2, j2);
    const int a = i1 + i2, b = j1 + j2, t = a + b;
    const int mu = t * (t + 1) / 2 + b;
    // only blocks with row block <= column block are formed (S is symmetric)
    const int lo = ((n >> 4) <= (n2 >> 4)) ? n : n2, hi = ((n >> 4) <= (n2 >> 4)) ? n2 : n;
    JtJ[idx] = S[(size_t)mu * 4096 + lo * 64 + hi];
}

__global__ void fill_ones_kernel(float* __restrict__ v, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) v[i] = 1.f;
}

__global__ void copy_plane_kernel(const float* __restrict__ src, float* __restrict__ dst, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) dst[i] = src[i];
}

// rhs[(n,m)] = S[mu(i_m, j_m)][n][q] = sum_{p in mask} P_m T_n I, where plane q
// of the band held I (column q of the Gram sums, q >= n, so the entry is formed)
__global__ void assemble_rhs(const double* __restrict__ S, int N, int M, int q, double* __restrict__ rhs) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= N * M) return;
    const int n = idx / M, m = idx % M;
    int t = 0;
    while ((t + 1) * (t + 2) / 2 <= m) ++t;
    const int j = m - t * (t + 1) / 2;
    rhs[idx] = S[(size_t)(t * (t + 1) / 2 + j) * 4096 + n * 64 + q];
}

// With a background polynomial the fit has one more "basis" whose response
// is the constant 1 (bg = sum_m b_m P_m * 1), so the same Gram sums give the
// background rows and columns of the normal matrix: plane N of the band is
// filled with ones.  With I and rhs given, one more plane holds I, and the
// Gram sums of the basis planes with it are the right-hand side
// rhs[(n,m)] = sum_p P_m T_n I of the normal equations.
int launch_normal_matrix(svconv_plan* p, const float* R, const float* I, const unsigned char* mask,
                         double* JtJ, double* rhs) {
    const int NF = p->N + p->bg;
    const bool want_rhs = (I != nullptr && rhs != nullptr);
    const int planes = NF + (want_rhs ? 1 : 0);
    if (planes > 64)
        return fail(SVCONV_EUNSUPPORTED,
                    "normal equations need N (+1 with a background, +1 with the right-hand side) <= 64");
    const int n_mu = (2 * p->d_s + 1) * (2 * p->d_s + 2) / 2;
    const int n_a = 2 * p->d_s + 1;                       // powers of xh
    const int cpr = (p->W + NM_PIX_CHUNK - 1) / NM_PIX_CHUNK;   // segments per row
    const size_t row_bytes = (size_t)planes * p->W * sizeof(float);
    int band = (int)(NM_BAND_BYTES / row_bytes);
    if (band < 8) band = 8;
    if (band > p->H) band = p->H;
    const size_t part_elems = (size_t)band * cpr * n_a * 4096;
    const size_t s_elems = (size_t)n_mu * 4096;
    const size_t tband_bytes = (size_t)band * row_bytes;
    const size_t nmpart_bytes = (part_elems + s_elems) * sizeof(double);
    // scratch of the normal matrix: allocated on its first call (grown when
    // a later call needs more), kept by the plan
    if (p->tband_bytes < tband_bytes || p->nmpart_bytes < nmpart_bytes) {
        if (p->dTband) (void)hipFree(p->dTband);
        if (p->dNMpart) (void)hipFree(p->dNMpart);
        p->dTband = nullptr;
        p->dNMpart = nullptr;
        p->tband_bytes = p->nmpart_bytes = 0;
        if (hipMalloc((void**)&p->dTband, tband_bytes) != hipSuccess ||
            hipMalloc((void**)&p->dNMpart, nmpart_bytes) != hipSuccess) {
            (void)hipGetLastError();
            if (p->dTband) (void)hipFree(p->dTband);
            p->dTband = nullptr;
            p->dNMpart = nullptr;
            return fail(SVCONV_ENOMEM, "normal-matrix scratch");
        }
        p->tband_bytes = tband_bytes;
        p->nmpart_bytes = nmpart_bytes;
    }
    double* S = p->dNMpart + part_elems;
    hipLaunchKernelGGL(zero_kernel, dim3(256), dim3(256), 0, p->stream, S, s_elems);
    int st = hip_status(hipGetLastError(), "zero_kernel");
    if (st) return st;

    ContractArgs c{};
    c.X = R;
    c.H = p->H;
    c.W = p->W;
    c.h = p->h;
    c.NF = p->N;
    c.M = p->M;
    c.d_s = p->d_s;
    c.coef = nullptr;
    c.beta = p->dBeta;
    c.ped = p->pedestal;
    c.I = nullptr;
    c.out = nullptr;
    double sx = 0, ox = 0, sy = 0, oy = 0;
    if (p->Wf > 1) { sx = 2.0 / (p->Wf - 1); ox = sx * p->x0 - 1.0; }
    if (p->Hf > 1) { sy = 2.0 / (p->Hf - 1); oy = sy * p->y0 - 1.0; }
    c.sx = sx; c.ox = ox; c.sy = sy; c.oy = oy;
    c.tout = p->dTband;
    // basis-form kernel with out == nullptr: coefficients are neither read nor used
    c.coef = reinterpret_cast<const float*>(p->dF32);
    const int nb = (p->N + 15) / 16;
    for (int y0 = 0; y0 < p->H; y0 += band) {
        const int rows = (y0 + band <= p->H) ? band : p->H - y0;
        c.y_begin = y0;
        c.n_rows = rows;
        if (sep_form(p)) {
            // basis responses through the separable factors
            SepArgs sa{};
            sa.X = R;
            sa.I = nullptr;
            sa.out = nullptr;
            sa.H = p->H;
            sa.W = p->W;
            sa.h = p->h;
            sa.ped = p->pedestal;
            sa.G = (int)p->sigmas.size();
            sa.fam = p->dSepFam;
            sa.f1d = p->dSep1d;
            sa.beta = p->dBeta;
            sa.coef = reinterpret_cast<const float*>(p->dF32);   // not read in this mode
            sa.M = p->M;
            sa.d_s = p->d_s;
            sa.sx = sx; sa.ox = ox; sa.sy = sy; sa.oy = oy;
            sa.y_begin = y0;
            sa.n_rows = rows;
            sa.tout = p->dTband;
            st = launch_contract_sep(sa, p->stream);
        } else {
            st = launch_contract_f32(c, p->dFragF32, nb, p->stream);
        }
        if (st) return st;
        const int band_px = rows * p->W;
        if (p->bg) {
            hipLaunchKernelGGL(fill_ones_kernel, dim3(1024), dim3(256), 0, p->stream,
                               p->dTband + (size_t)p->N * band_px, band_px);
            st = hip_status(hipGetLastError(), "fill_ones_kernel");
            if (st) return st;
        }
        if (want_rhs) {
            hipLaunchKernelGGL(copy_plane_kernel, dim3(1024), dim3(256), 0, p->stream,
                               I + (size_t)y0 * p->W, p->dTband + (size_t)NF * band_px, band_px);
            st = hip_status(hipGetLastError(), "copy_plane_kernel");
            if (st) return st;
        }
        const int segs = rows * cpr;
        hipLaunchKernelGGL(gram_kernel, dim3(n_a, segs), dim3(64 * GRAM_WAVES), 0, p->stream, p->dTband, planes,
                           band_px, y0, p->W, p->H, p->h, cpr, mask, sx, ox, n_a, p->dNMpart);
        st = hip_status(hipGetLastError(), "gram_kernel");
        if (st) return st;
        hipLaunchKernelGGL(gram_reduce, dim3(4096 / 256, n_a), dim3(256), 0, p->stream,
                           p->dNMpart, segs, cpr, n_a, y0, sy, oy, S);
        st = hip_status(hipGetLastError(), "gram_reduce");
        if (st) return st;
    }
    const int NM = NF * p->M;
    hipLaunchKernelGGL(assemble_jtj, dim3((NM * NM + 255) / 256), dim3(256), 0, p->stream, S, NF,
                       p->M, JtJ);
    st = hip_status(hipGetLastError(), "assemble_jtj");
    if (st || !want_rhs) return st;
    hipLaunchKernelGGL(assemble_rhs, dim3((NM + 255) / 256), dim3(256), 0, p->stream, S, NF, p->M, NF, rhs);
    return hip_status(hipGetLastError(), "assemble_rhs");
}

// -------------------------------------------------------- Cholesky ----

// Right-looking in-place factorisation by one workgroup; A stays in global
// memory (at most 1024 x 1024 doubles, resident in L2).  status[0] becomes
// the first non-positive pivot index + 1 (0 = SPD).
__global__ __launch_bounds__(1024) void cholesky_kernel(double* __restrict__ A, int n,
                                                        int* __restrict__ status) {
    __shared__ int bad;
    __shared__ double piv;
    const int tid = threadIdx.x;
    if (tid == 0) bad = 0;
    __syncthreads();
    for (int jc = 0; jc < n; ++jc) {
        if (tid == 0) {
            const double d = A[(size_t)jc * n + jc];
            if (!(d > 0.0) || !isfinite(d)) {
                bad = jc + 1;
                piv = 1.0;
            } else {
                piv = sqrt(d);
                A[(size_t)jc * n + jc] = piv;
            }
        }
        __syncthreads();
        if (bad) break;
        const double inv = 1.0 / piv;
        for (int i = jc + 1 + tid; i < n; i += 1024) A[(size_t)i * n + jc] *= inv;
        __syncthreads();
        // trailing update of the lower triangle: A[i][c] -= L[i][jc] L[c][jc], jc < c <= i
        const int m = n - jc - 1;
        const long cnt = (long)m * (m + 1) / 2;
        for (long q = tid; q < cnt; q += 1024) {
            // row-major enumeration of the lower triangle of an m x m block
            long i = (long)((sqrt(8.0 * q + 1.0) - 1.0) * 0.5);
            while (i * (i + 1) / 2 > q) --i;
            while ((i + 1) * (i + 2) / 2 <= q) ++i;
            const long c = q - i * (i + 1) / 2;
            const int ii = jc + 1 + (int)i, cc = jc + 1 + (int)c;
            A[(size_t)ii * n + cc] -= A[(size_t)ii * n + jc] * A[(size_t)cc * n + jc];
        }
        __syncthreads();
    }
    __syncthreads();
    if (!bad) {
        for (long q = tid; q < (long)n * n; q += 1024) {
            const int i = (int)(q / n), c = (int)(q % n);
            if (c > i) A[q] = 0.0;
        }
    }
    if (tid == 0) status[0] = bad;
}

// Blocked right-looking factorisation for larger matrices: for each block
// column k0 of width CH_NB, one workgroup factors the diagonal block in LDS
// and solves the panel below it (L21 = A21 L11^-T), then one workgroup per
// 32 x 32 tile of the trailing lower triangle applies A22 -= L21 L21^T.
constexpr int CH_NB = 32;

__global__ __launch_bounds__(256) void chol_panel_kernel(double* __restrict__ A, int n, int k0,
                                                         int* __restrict__ status) {
    __shared__ double L[CH_NB][CH_NB + 1];
    __shared__ int bad;
    const int tid = threadIdx.x;
    const int nb = min(CH_NB, n - k0);
    for (int q = tid; q < nb * nb; q += 256) {
        const int r = q / nb, c = q - r * nb;
        L[r][c] = A[(size_t)(k0 + r) * n + k0 + c];
    }
    if (tid == 0) bad = status[0];
    __syncthreads();
    for (int j = 0; j < nb; ++j) {
        if (tid == 0) {
            double d = L[j][j];
            if (!(d > 0.0) || !isfinite(d)) {
                if (!bad) bad = k0 + j + 1;
                d = 1.0;
            }
            L[j][j] = sqrt(d);
        }
        __syncthreads();
        const double inv = 1.0 / L[j][j];
        for (int i = j + 1 + tid; i < nb; i += 256) L[i][j] *= inv;
        __syncthreads();
        const int m = nb - j - 1;
        for (int q = tid; q < m * m; q += 256) {
            const int i = j + 1 + q / m, c = j + 1 + q % m;
            if (c <= i) L[i][c] -= L[i][j] * L[c][j];
        }
        __syncthreads();
    }
    for (int q = tid; q < nb * nb; q += 256) {
        const int r = q / nb, c = q - r * nb;
        A[(size_t)(k0 + r) * n + k0 + c] = (c <= r) ? L[r][c] : 0.0;
    }
    // panel rows below: x L11^T = a, forward substitution over the block's
    // columns on the row held in registers; the empty asm with a memory clobber
    // keeps the compiler from hoisting all of L11 into registers across rows
    for (int i = k0 + nb + tid; i < n; i += 256) {
        asm volatile("" ::: "memory");
        double x[CH_NB];
        double* row = A + (size_t)i * n + k0;
#pragma unroll
        for (int c = 0; c < CH_NB; ++c) {
            if (c < nb) {
                double s = row[c];
#pragma unroll
                for (int t = 0; t < c; ++t) s -= x[t] * L[c][t];
                x[c] = s / L[c][c];
                row[c] = x[c];
            }
        }
    }
    if (tid == 0) status[0] = bad;
}

// A22 -= L21 L21^T on the lower triangle; block b is tile (ti, tj), tj <= ti
__global__ __launch_bounds__(256) void chol_update_kernel(double* __restrict__ A, int n, int k0,
                                                          int nb) {
    __shared__ double Li[CH_NB][CH_NB + 1], Lj[CH_NB][CH_NB + 1];
    const int b = blockIdx.x;
    int ti = (int)((sqrt(8.0 * b + 1.0) - 1.0) * 0.5);
    while (ti * (ti + 1) / 2 > b) --ti;
    while ((ti + 1) * (ti + 2) / 2 <= b) ++ti;
    const int tj = b - ti * (ti + 1) / 2;
    const int k1 = k0 + nb;
    const int r0 = k1 + 32 * ti, c0 = k1 + 32 * tj;
    const int tid = threadIdx.x;
    for (int q = tid; q < 32 * nb; q += 256) {
        const int r = q / nb, c = q - r * nb;
        Li[r][c] = (r0 + r < n) ? A[(size_t)(r0 + r) * n + k0 + c] : 0.0;
        Lj[r][c] = (c0 + r < n) ? A[(size_t)(c0 + r) * n + k0 + c] : 0.0;
    }
    __syncthreads();
    const int cc = tid & 31, rb = tid >> 5;     // column, first of 4 rows (stride 8)
    for (int rr = rb; rr < 32; rr += 8) {
        const int gi = r0 + rr, gj = c0 + cc;
        if (gi < n && gj < n && gj <= gi) {
            double s = 0.0;
            for (int t = 0; t < nb; ++t) s = fma(Li[rr][t], Lj[cc][t], s);
            A[(size_t)gi * n + gj] -= s;
        }
    }
}

__global__ void chol_zero_upper(double* __restrict__ A, int n) {
    const size_t total = (size_t)n * n;
    for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < total;
         q += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(q / n), c = (int)(q % n);
        if (c > i) A[q] = 0.0;
    }
}

__global__ void chol_status_clear(int* status) {
    if (threadIdx.x == 0) status[0] = 0;
}

int launch_cholesky(svconv_plan* p, double* A, int n) {
    int st = SVCONV_OK;
    if (n <= 64) {
        hipLaunchKernelGGL(cholesky_kernel, dim3(1), dim3(1024), 0, p->stream, A, n, p->dStatus);
        st = hip_status(hipGetLastError(), "cholesky_kernel");
    } else {
        hipLaunchKernelGGL(chol_status_clear, dim3(1), dim3(64), 0, p->stream, p->dStatus);
        st = hip_status(hipGetLastError(), "chol_status_clear");
        for (int k0 = 0; k0 < n && !st; k0 += CH_NB) {
            const int nb = (n - k0) < CH_NB ? (n - k0) : CH_NB;
            hipLaunchKernelGGL(chol_panel_kernel, dim3(1), dim3(256), 0, p->stream, A, n, k0, p->dStatus);
            st = hip_status(hipGetLastError(), "chol_panel_kernel");
            const int rest = n - k0 - nb;
            if (!st && rest > 0) {
                const int nt = (rest + 31) / 32;
                hipLaunchKernelGGL(chol_update_kernel, dim3(nt * (nt + 1) / 2), dim3(256), 0, p->stream,
                                   A, n, k0, nb);
                st = hip_status(hipGetLastError(), "chol_update_kernel");
            }
        }
        if (!st) {
            hipLaunchKernelGGL(chol_zero_upper, dim3(256), dim3(256), 0, p->stream, A, n);
            st = hip_status(hipGetLastError(), "chol_zero_upper");
        }
    }
    if (st) return st;
    int bad = 0;
    st = hip_status(hipMemcpyAsync(&bad, p->dStatus, sizeof(int), hipMemcpyDeviceToHost, p->stream),
                    "copy status");
    if (!st) st = hip_status(hipStreamSynchronize(p->stream), "hipStreamSynchronize");
    if (st) return st;
    if (bad) return fail(SVCONV_ENOTSPD, "pivot " + std::to_string(bad - 1) + " is not positive");
    return SVCONV_OK;
}

// x = L^-T L^-1 rhs by blocked substitutions in one workgroup of 1024
// threads.  Per block of 32 unknowns, one wave solves the 32 x 32 triangle
// (each unknown broadcast across the lanes, the diagonal's reciprocals formed
// first); then every thread folds the block's unknowns into the right-hand
// side entries still to be solved (right-looking): one row of the panel per
// thread in the forward pass (32 independent loads of contiguous doubles),
// one column per thread in the backward pass (loads coalesced across the
// wave).  So each block waits on memory once.  v holds the right-hand side,
// then the solution.
constexpr int CS_B = 32;

__global__ __launch_bounds__(1024) void chol_solve_kernel(const double* __restrict__ L,
                                                          const double* __restrict__ rhs,
                                                          double* __restrict__ x, int n) {
    extern __shared__ double v[];   // n doubles
    const int tid = threadIdx.x;
    for (int i = tid; i < n; i += 1024) v[i] = rhs[i];
    __syncthreads();
    const int nblk = (n + CS_B - 1) / CS_B;
    // forward: L y = b
    for (int kb = 0; kb < nblk; ++kb) {
        const int j0 = kb * CS_B, nb = min(CS_B, n - j0);
        if (tid < 64) {
            // lane t < nb: row j0 + t of the triangle, loaded into registers first
            const int t = tid;
            const bool live = t < nb;
            const double* Lt = L + (size_t)(j0 + (live ? t : 0)) * n + j0;
            double l[CS_B];
#pragma unroll
            for (int j = 0; j < CS_B; ++j) l[j] = (live && j < nb) ? Lt[j] : 0.0;
            const double inv = live ? 1.0 / Lt[t] : 0.0;
            double acc = live ? v[j0 + t] : 0.0;
#pragma unroll
            for (int j = 0; j < CS_B; ++j) {
                if (j < nb) {
                    const double yj = __shfl(acc, j) * __shfl(inv, j);
                    if (t > j) acc = fma(-l[j], yj, acc);
                    if (t == j) acc = yj;
                }
            }
            if (live) v[j0 + t] = acc;
        }
        __syncthreads();
        // rows below the block: v[i] -= L[i][j0 .. j0 + nb) y
        for (int i = j0 + nb + tid; i < n; i += 1024) {
            const double* Li = L + (size_t)i * n + j0;
            double s = 0.0;
            if (nb == CS_B) {
                // a full block: the row's loads issued together
                double l[CS_B];
#pragma unroll
                for (int c = 0; c < CS_B; ++c) l[c] = Li[c];
#pragma unroll
                for (int c = 0; c < CS_B; ++c) s = fma(l[c], v[j0 + c], s);
            } else {
                for (int c = 0; c < nb; ++c) s = fma(Li[c], v[j0 + c], s);
            }
            v[i] -= s;
        }
        __syncthreads();
    }
    // backward: L^T x = y
    for (int kb = nblk - 1; kb >= 0; --kb) {
        const int j0 = kb * CS_B, nb = min(CS_B, n - j0);
        if (tid < 64) {
            // lane t < nb: column j0 + t of the triangle, loaded into registers first
            const int t = tid;
            const bool live = t < nb;
            const double* Lc = L + (size_t)j0 * n + j0 + (live ? t : 0);
            double l[CS_B];
#pragma unroll
            for (int j = 0; j < CS_B; ++j) l[j] = (live && j < nb) ? Lc[(size_t)j * n] : 0.0;
            const double inv = live ? 1.0 / Lc[(size_t)t * n] : 0.0;
            double acc = live ? v[j0 + t] : 0.0;
#pragma unroll
            for (int j = CS_B - 1; j >= 0; --j) {
                if (j < nb) {
                    const double xj = __shfl(acc, j) * __shfl(inv, j);
                    if (t < j) acc = fma(-l[j], xj, acc);
                    if (t == j) acc = xj;
                }
            }
            if (live) v[j0 + t] = acc;
        }
        __syncthreads();
        // columns left of the block: v[c] -= sum_r L[j0 + r][c] x[j0 + r]
        for (int c = tid; c < j0; c += 1024) {
            double s = 0.0;
            if (nb == CS_B) {
                double l[CS_B];
#pragma unroll
                for (int r = 0; r < CS_B; ++r) l[r] = L[(size_t)(j0 + r) * n + c];
#pragma unroll
                for (int r = 0; r < CS_B; ++r) s = fma(l[r], v[j0 + r], s);
            } else {
                for (int r = 0; r < nb; ++r) s = fma(L[(size_t)(j0 + r) * n + c], v[j0 + r], s);
            }
            v[c] -= s;
        }
        __syncthreads();
    }
    for (int i = tid; i < n; i += 1024) x[i] = v[i];
}

int launch_cholesky_solve(svconv_plan* p, const double* L, const double* rhs, double* x, int n) {
    hipLaunchKernelGGL(chol_solve_kernel, dim3(1), dim3(1024), (size_t)n * sizeof(double), p->stream,
                       L, rhs, x, n);
    return hip_status(hipGetLastError(), "chol_solve_kernel");
}

// --------------------------------------------------------- updates ----

__global__ void scale_kernel(double* v, double s, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) v[i] *= s;
}

__global__ void copy_a_kernel(const double* a64, float* a32, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a32[i] = (float)a64[i];
}

// a64 -= delta, a32 = float(a64), norm = ||delta||_2 (one workgroup)
__global__ __launch_bounds__(1024) void gn_update_kernel(const double* __restrict__ delta,
                                                         double* __restrict__ a64,
                                                         float* __restrict__ a32, int n,
                                                         double* __restrict__ norm) {
    __shared__ double red[1024];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 1024) {
        const double d = delta[i];
        const double v = a64[i] - d;
        a64[i] = v;
        a32[i] = (float)v;
        s += d * d;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *norm = sqrt(red[0]);
}

int launch_scale(svconv_plan* p, double* v, double s, int n) {
    hipLaunchKernelGGL(scale_kernel, dim3((n + 255) / 256), dim3(256), 0, p->stream, v, s, n);
    return hip_status(hipGetLastError(), "scale_kernel");
}

int launch_copy_a(svconv_plan* p, const double* a64, float* a32, int n) {
    hipLaunchKernelGGL(copy_a_kernel, dim3((n + 255) / 256), dim3(256), 0, p->stream, a64, a32, n);
    return hip_status(hipGetLastError(), "copy_a_kernel");
}

// g = A a - rhs (the half-gradient of the loss, J^T D, from the normal
// equations): one wave per row of the symmetric A, lanes over its columns.
// The dot product is compensated (error-free products and sums, Ogita, Rump
// and Oishi's Dot2): g is then as accurate as if formed in twice the float64
// precision and rounded once, which iterative refinement needs to converge
// past cond(A) eps (A a and rhs nearly cancel at the solution).
__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
#pragma clang fp contract(off)
    s = a + b;
    const double bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

__device__ __forceinline__ void two_prod(double a, double b, double& p, double& e) {
#pragma clang fp contract(off)
    p = a * b;
    e = fma(a, b, -p);
}

__global__ __launch_bounds__(256) void ls_grad_kernel(const double* __restrict__ A,
                                                      const double* __restrict__ a,
                                                      const double* __restrict__ rhs, int n,
                                                      double* __restrict__ g) {
#pragma clang fp contract(off)
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (row >= n) return;
    const double* Ar = A + (size_t)row * n;
    double s = 0.0, c = 0.0;   // sum and its accumulated error terms
    for (int k = lane; k < n; k += 64) {
        double p, pe, t, te;
        two_prod(Ar[k], a[k], p, pe);
        two_sum(s, p, t, te);
        s = t;
        c += te + pe;
    }
    for (int o = 32; o > 0; o >>= 1) {
        const double so = __shfl_xor(s, o), co = __shfl_xor(c, o);
        double t, te;
        two_sum(s, so, t, te);
        s = t;
        c += co + te;
    }
    if (lane == 0) {
        double t, te;
        two_sum(s, -rhs[row], t, te);
        g[row] = t + (c + te);
    }
}

int launch_ls_grad(svconv_plan* p, const double* A, const double* a64, const double* rhs, double* g, int n) {
    hipLaunchKernelGGL(ls_grad_kernel, dim3((n + 3) / 4), dim3(256), 0, p->stream, A, a64, rhs, n, g);
    return hip_status(hipGetLastError(), "ls_grad_kernel");
}

int launch_gn_update(svconv_plan* p, const double* delta, double* a64, float* a32, int n) {
    // the step norm lands right after the loss scalar in the plan's vector scratch
    double* norm = p->dVec + 2 * (size_t)n + 1;
    hipLaunchKernelGGL(gn_update_kernel, dim3(1), dim3(1024), 0, p->stream, delta, a64, a32, n, norm);
    return hip_status(hipGetLastError(), "gn_update_kernel");
}

}  // namespace svc
