// Adjoint of the difference image in the coefficients a[n][m].
//
// D(p) = sum_n sum_m a[n][m] P_m(p) T_n(p) - I(p) with
// T_n(p) = sum_tap F_n[tap] R(p + off(tap)), so for G = dL/dD
//
//   dL/da[n][m] = sum_p G(p) P_m(p) T_n(p) = sum_tap F_n[tap] Q_m[tap],
//   Q_m[tap]    = sum_p G(p) P_m(p) R(p + off(tap)).
//
// Q is an (M x pixels) . (pixels x taps) product: the reduction runs over
// all pixels and the output is only M x k^2, the shape of a convolution
// weight gradient.  It runs on the float32 matrix cores
// (v_mfma_f32_16x16x4_f32: 4 pixels x 16 taps x 16 terms per instruction)
// with the patches read from an LDS tile of R, per-tile partial sums in
// float32 and everything after in float64: per-workgroup totals, the
// deterministic reduction over workgroups and the final F . Q^T.  Compared
// with recomputing the N basis responses T_n this does M instead of N
// filters' worth of multiply-adds.
#include "internal.hpp"

namespace svc {

typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int AQ_TW = 64;     // pixel tile: 64 x 16
constexpr int AQ_TH = 16;
constexpr int AQ_WAVES = 4;
constexpr size_t AQ_SCRATCH_BYTES = (size_t)96 << 20;   // cap of the partial-sum scratch

struct AdjointQGeometry {
    int mb, tbw;           // 16-term blocks, tap blocks per wave
    int n_tap_blocks, n_tg, taps_pad;
    int rows, cols, pitch;
    int tiles_x, n_tiles, n_wg;
    size_t lds_bytes;
};

static AdjointQGeometry aq_geometry(int H, int W, int k, int M) {
    AdjointQGeometry g;
    g.mb = (M + 15) / 16;
    g.tbw = g.mb == 1 ? 16 : 8;
    g.n_tap_blocks = (k * k + 15) / 16;
    g.n_tg = (g.n_tap_blocks + AQ_WAVES * g.tbw - 1) / (AQ_WAVES * g.tbw);
    g.taps_pad = g.n_tg * AQ_WAVES * g.tbw * 16;
    g.rows = AQ_TH + k - 1;
    g.cols = AQ_TW + k - 1;
    g.pitch = g.cols;
    g.tiles_x = (W + AQ_TW - 1) / AQ_TW;
    g.n_tiles = g.tiles_x * ((H + AQ_TH - 1) / AQ_TH);
    const size_t per_wg = (size_t)16 * g.mb * g.taps_pad * sizeof(double);
    int cap = (int)(AQ_SCRATCH_BYTES / per_wg);
    if (cap < 1) cap = 1;
    g.n_wg = g.n_tiles < 512 ? g.n_tiles : 512;
    if (g.n_wg > cap) g.n_wg = cap;
    // R tile plus its halo, then the G tile
    g.lds_bytes = ((size_t)g.rows * g.pitch + AQ_TW * AQ_TH) * sizeof(float);
    return g;
}

size_t adjoint_scratch_doubles(int H, int W, int k, int M) {
    const AdjointQGeometry g = aq_geometry(H, W, k, M);
    return (size_t)g.n_wg * 16 * g.mb * g.taps_pad + (size_t)16 * g.mb * g.taps_pad;
}

// x^e for 0 <= e <= 7 from the binary digits of e (no branches)
__device__ __forceinline__ double pow_q(double x, double x2, double x4, int e) {
    return ((e & 1) ? x : 1.0) * ((e & 2) ? x2 : 1.0) * ((e & 4) ? x4 : 1.0);
}

template <int MB, int TBW>
__global__ __launch_bounds__(256, 2) void adjoint_q_kernel(
    const float* __restrict__ R, const float* __restrict__ G, int H, int W, int h, int k, int M,
    double sx, double ox, double sy, double oy, int tiles_x, int n_tiles, int n_wg, int taps_pad,
    int pitch, int rows, int cols, double* __restrict__ part) {
    extern __shared__ __align__(16) float tile[];
    float* gtile = tile + rows * pitch;   // G of the tile's AQ_TH x AQ_TW pixels
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int kq = lane >> 4, j = lane & 15;
    const int kk = k * k;

    // LDS offsets of this lane's taps, tap = 16 (T0 + t) + j
    const int T0 = (blockIdx.y * AQ_WAVES + w) * TBW;
    int off[TBW];
#pragma unroll
    for (int t = 0; t < TBW; ++t) {
        const int tau = 16 * (T0 + t) + j;
        off[t] = tau < kk ? (tau / k) * pitch + (tau % k) : 0;
    }
    // spatial term carried by this lane in the A operand: m = 16 mb + j
    int ei[MB], ej[MB];
    bool mv[MB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
        const int m = 16 * mb + j;
        int tt = 0;
        while ((tt + 1) * (tt + 2) / 2 <= m) ++tt;
        ej[mb] = m - tt * (tt + 1) / 2;
        ei[mb] = tt - ej[mb];
        mv[mb] = m < M;
    }

    double tot[MB][TBW][4];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int t = 0; t < TBW; ++t)
#pragma unroll
            for (int e = 0; e < 4; ++e) tot[mb][t][e] = 0.0;

    for (int ti = blockIdx.x; ti < n_tiles; ti += n_wg) {
        const int X0 = (ti % tiles_x) * AQ_TW;
        const int Y0 = (ti / tiles_x) * AQ_TH;
        __syncthreads();   // the previous tile's reads are done
        // R with its halo and G: the loads of AQ_SB elements per thread go
        // out together from clamped addresses, the masks apply at the store
        constexpr int AQ_SB = 8;
        for (int q0 = tid; q0 < rows * cols; q0 += 256 * AQ_SB) {
            float v[AQ_SB];
#pragma unroll
            for (int sb = 0; sb < AQ_SB; ++sb) {
                const int q = q0 + 256 * sb, r = q / cols, c = q - r * cols;
                const int gy = Y0 - h + r, gx = X0 - h + c;
                v[sb] = R[(size_t)(gy < 0 ? 0 : (gy < H ? gy : H - 1)) * W + (gx < 0 ? 0 : (gx < W ? gx : W - 1))];
            }
#pragma unroll
            for (int sb = 0; sb < AQ_SB; ++sb) {
                const int q = q0 + 256 * sb, r = q / cols, c = q - r * cols;
                const int gy = Y0 - h + r, gx = X0 - h + c;
                if (q < rows * cols) tile[r * pitch + c] = (gy >= 0 && gy < H && gx >= 0 && gx < W) ? v[sb] : 0.f;
            }
        }
        {
            float v[AQ_TW * AQ_TH / 256];
#pragma unroll
            for (int sb = 0; sb < AQ_TW * AQ_TH / 256; ++sb) {
                const int p = tid + 256 * sb, x = X0 + p % AQ_TW, y = Y0 + p / AQ_TW;
                v[sb] = G[(size_t)(y < H ? y : H - 1) * W + (x < W ? x : W - 1)];
            }
#pragma unroll
            for (int sb = 0; sb < AQ_TW * AQ_TH / 256; ++sb) {
                const int p = tid + 256 * sb, x = X0 + p % AQ_TW, y = Y0 + p / AQ_TW;
                gtile[p] = (x < W && y < H) ? v[sb] : 0.f;
            }
        }
        __syncthreads();

        f4 acc[MB][TBW];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int t = 0; t < TBW; ++t) acc[mb][t] = f4{0.f, 0.f, 0.f, 0.f};

        for (int s = 0; s < AQ_TW * AQ_TH / 4; ++s) {
            const int p = 4 * s + kq;
            const int px = p % AQ_TW, py = p / AQ_TW;
            const int x = X0 + px, y = Y0 + py;
            const double gv = (double)gtile[p];
            const double xh = sx * x + ox, yh = sy * y + oy;
            const double xh2 = xh * xh, xh4 = xh2 * xh2, yh2 = yh * yh, yh4 = yh2 * yh2;
            float af[MB];
#pragma unroll
            for (int mb = 0; mb < MB; ++mb)
                af[mb] = mv[mb] ? (float)(gv * pow_q(xh, xh2, xh4, ei[mb]) * pow_q(yh, yh2, yh4, ej[mb]))
                                : 0.f;
            const float* tb = tile + py * pitch + px;
#pragma unroll
            for (int t = 0; t < TBW; ++t) {
                const float xb = tb[off[t]];
#pragma unroll
                for (int mb = 0; mb < MB; ++mb)
                    acc[mb][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[mb], xb, acc[mb][t], 0, 0, 0);
            }
        }
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int t = 0; t < TBW; ++t)
#pragma unroll
                for (int e = 0; e < 4; ++e) tot[mb][t][e] += (double)acc[mb][t][e];
    }

    // lane (kq, j) holds Q[m = 16 mb + 4 kq + e][tap = 16 (T0 + t) + j]
    double* dst = part + (size_t)blockIdx.x * (16 * MB) * taps_pad;
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int t = 0; t < TBW; ++t)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int m = 16 * mb + 4 * kq + e;
                const int tau = 16 * (T0 + t) + j;
                dst[(size_t)m * taps_pad + tau] = tot[mb][t][e];
            }
}

// Q[m][tap] = sum over workgroups of the partials (fixed order).
__global__ void adjoint_q_reduce(const double* __restrict__ part, int n_wg, int rows_m,
                                 int taps_pad, double* __restrict__ Q) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= rows_m * taps_pad) return;
    double s = 0.0;
    for (int b = 0; b < n_wg; ++b) s += part[(size_t)b * rows_m * taps_pad + idx];
    Q[idx] = s;
}

// ga[n][m] = sum_tap F_n[tap] Q_m[tap] in float64, one wave per (n, m).
__global__ void adjoint_a_final(const double* __restrict__ F64, const double* __restrict__ Q,
                                int N, int M, int kk, int taps_pad, double* __restrict__ ga) {
    const int nm = blockIdx.x;
    const int n = nm / M, m = nm % M;
    double s = 0.0;
    for (int t = threadIdx.x; t < kk; t += 64) s += F64[(size_t)n * kk + t] * Q[(size_t)m * taps_pad + t];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (threadIdx.x == 0) ga[nm] = s;
}

int launch_adjoint_a(svconv_plan* p, const float* R, const float* gD, double* ga) {
    // a plan in the separable form takes the adjoint through the same factors
    // (when its per-round moments fit in LDS; otherwise the product below)
    if (sep_form(p) && sep_adjoint_supported(p))
        return launch_adjoint_a_sep(p, R, gD, ga);
    const AdjointQGeometry g = aq_geometry(p->H, p->W, p->k, p->M);
    if (!p->dQpart) return fail(SVCONV_ENOMEM, "adjoint scratch missing");
    double sx = 0, ox = 0, sy = 0, oy = 0;
    if (p->Wf > 1) { sx = 2.0 / (p->Wf - 1); ox = sx * p->x0 - 1.0; }
    if (p->Hf > 1) { sy = 2.0 / (p->Hf - 1); oy = sy * p->y0 - 1.0; }
    double* Q = p->dQpart + (size_t)g.n_wg * 16 * g.mb * g.taps_pad;
    dim3 grid(g.n_wg, g.n_tg);
    if (g.mb == 1)
        hipLaunchKernelGGL((adjoint_q_kernel<1, 16>), grid, dim3(256), g.lds_bytes, p->stream, R, gD,
                           p->H, p->W, p->h, p->k, p->M, sx, ox, sy, oy, g.tiles_x, g.n_tiles,
                           g.n_wg, g.taps_pad, g.pitch, g.rows, g.cols, p->dQpart);
    else if (g.mb == 2)
        hipLaunchKernelGGL((adjoint_q_kernel<2, 8>), grid, dim3(256), g.lds_bytes, p->stream, R, gD,
                           p->H, p->W, p->h, p->k, p->M, sx, ox, sy, oy, g.tiles_x, g.n_tiles,
                           g.n_wg, g.taps_pad, g.pitch, g.rows, g.cols, p->dQpart);
    else
        return fail(SVCONV_EUNSUPPORTED, "adjoint in a needs M <= 32");
    int st = hip_status(hipGetLastError(), "adjoint_q_kernel");
    if (st) return st;
    const int rows_m = 16 * g.mb;
    const int total = rows_m * g.taps_pad;
    hipLaunchKernelGGL(adjoint_q_reduce, dim3((total + 255) / 256), dim3(256), 0, p->stream,
                       p->dQpart, g.n_wg, rows_m, g.taps_pad, Q);
    st = hip_status(hipGetLastError(), "adjoint_q_reduce");
    if (st) return st;
    hipLaunchKernelGGL(adjoint_a_final, dim3(p->N * p->M), dim3(64), 0, p->stream, p->dF64, Q,
                       p->N, p->M, p->k * p->k, g.taps_pad, ga);
    return hip_status(hipGetLastError(), "adjoint_a_final");
}

}  // namespace svc
