// Regrouped contraction for small kernels on the vector units.
//
// D = sum_m P_m (Kt_m (x) R) - I (Eq. 1 with Eq. 2 regrouped: P_m depends
// only on the output pixel, so the M kernels Kt_m = sum_n a[n][m] B_n carry
// all of the coefficients).  For the Dirac delta basis (Sec. 2) Kt_m is the
// coefficient array itself, Kt_m[u,v] = a[n(u,v)][m], so the taps are read
// straight from a and no per-call table is built.
//
// With k <= 9 taps per axis the contraction is 2 M k^2 FLOP per pixel (588 at
// the paper's 7 x 7, second-order case), too little work per byte for the
// matrix cores' padded 16-filter blocks to pay: plain float32 FMAs with the
// taps in scalar registers (uniform over the wave) and the staged tile in
// LDS.  Each thread owns 8 consecutive output rows of one column; per kernel
// row it sums the k taps of each spatial term in float32 and adds that row
// sum into a float64 total, which keeps the float32 rounding to one kernel
// row's worth.  The pedestal restore s sum_m gamma_m P_m and the subtraction
// of I are in float64.
//
// Workgroup: 256 threads, output tile 64 x 32 (4 row groups of 8 rows).
#include "internal.hpp"
#include "sep_fold.hpp"

namespace svc {

constexpr int DR_TW = 64, DR_TH = 32, DR_NT = 256, DR_RPT = 8;

// DFB: tap (m, dv, du) = a[(k^2 - 1 - (dv k + du)) M + m] (the delta basis in
// correlation orientation); otherwise taps[m][dv][du] (the regrouped filters).
template <int H, int DS, bool DFB>
__global__ __launch_bounds__(DR_NT) void contract_direct_kernel(DirectArgs a) {
    constexpr int K = 2 * H + 1;
    constexpr int M = (DS + 1) * (DS + 2) / 2;
    constexpr int SR = DR_TH + 2 * H, SC = DR_TW + 2 * H;
    __shared__ float tile[SR][SC];
    __shared__ double gam_s[M];

    const int tid = threadIdx.x, c = tid & 63, rg = tid >> 6;
    const int tx = blockIdx.x % a.tiles_x, ty = blockIdx.x / a.tiles_x;
    const int X0 = tx * DR_TW, Y0 = ty * DR_TH;
    const cptr<float> tp = as_const(a.taps);
    auto tap = [&](int m, int t) -> float { return DFB ? tp[(K * K - 1 - t) * M + m] : tp[m * K * K + t]; };

    // stage R - s; R = 0 outside the image.  Every sample is loaded from a
    // clamped, in-image address and none conditionally, so that all loads are
    // in flight together; the image mask applies when storing.
    constexpr int SITER = (SR * SC + DR_NT - 1) / DR_NT;
    float sv[SITER];
#pragma unroll
    for (int i = 0; i < SITER; ++i) {
        const int q = min(tid + i * DR_NT, SR * SC - 1);
        const int r = q / SC, cc = q - r * SC;
        const int gy = min(max(Y0 - H + r, 0), a.H - 1), gx = min(max(X0 - H + cc, 0), a.W - 1);
        sv[i] = a.X[(size_t)gy * a.W + gx];
    }
#pragma unroll
    for (int i = 0; i < SITER; ++i) {
        const int q = tid + i * DR_NT;
        if (q < SR * SC) {
            const int r = q / SC, cc = q - r * SC;
            const int gy = Y0 - H + r, gx = X0 - H + cc;
            const float x = (gy >= 0 && gy < a.H && gx >= 0 && gx < a.W) ? sv[i] : 0.f;
            tile[r][cc] = x - a.ped;
        }
    }
    // pedestal sums gamma_m = sum of Kt_m's taps (float64)
    if (tid < M) {
        double s = 0.0;
        for (int t = 0; t < K * K; ++t) s += (double)tap(tid, t);
        gam_s[tid] = s;
    }
    __syncthreads();

    double tot[DR_RPT][M];
#pragma unroll
    for (int o = 0; o < DR_RPT; ++o)
#pragma unroll
        for (int m = 0; m < M; ++m) tot[o][m] = 0.0;

#pragma unroll 1
    for (int dv0 = 0; dv0 < K; ++dv0) {
        // the kernel row's taps: uniform addresses with constant offsets, so they
        // arrive by scalar loads
        const int dv = __builtin_amdgcn_readfirstlane(dv0);
        float tv[K][M];
        if constexpr (DFB) {
            const cptr<float> row = tp + (K * K - K - dv * K) * M;   // du = K - 1 at the lowest address
#pragma unroll
            for (int du = 0; du < K; ++du)
#pragma unroll
                for (int m = 0; m < M; ++m) tv[du][m] = row[(K - 1 - du) * M + m];
        } else {
            const cptr<float> row = tp + dv * K;
#pragma unroll
            for (int du = 0; du < K; ++du)
#pragma unroll
                for (int m = 0; m < M; ++m) tv[du][m] = row[m * K * K + du];
        }
#pragma unroll
        for (int o = 0; o < DR_RPT; ++o) {
            const float* row = &tile[DR_RPT * rg + o + dv][c];
            float racc[M];
#pragma unroll
            for (int m = 0; m < M; ++m) racc[m] = 0.f;
#pragma unroll
            for (int du = 0; du < K; ++du) {
                const float smp = row[du];
#pragma unroll
                for (int m = 0; m < M; ++m) racc[m] = fmaf(tv[du][m], smp, racc[m]);
            }
#pragma unroll
            for (int m = 0; m < M; ++m) tot[o][m] += (double)racc[m];
        }
    }

    const int x = X0 + c;
    if (x >= a.W) return;
    // I at this thread's pixels, all requested at once from clamped addresses
    // (without I, R stands in for the loads)
    float iv[DR_RPT];
    {
        const float* ip = a.I ? a.I : a.X;
#pragma unroll
        for (int o = 0; o < DR_RPT; ++o) iv[o] = ip[(size_t)min(Y0 + DR_RPT * rg + o, a.H - 1) * a.W + x];
    }
    const double xh = a.sx * x + a.ox;
    double xp[DS + 1];
    xp[0] = 1.0;
#pragma unroll
    for (int q = 1; q <= DS; ++q) xp[q] = xp[q - 1] * xh;
#pragma unroll
    for (int o = 0; o < DR_RPT; ++o) {
        const int y = Y0 + DR_RPT * rg + o;
        if (y >= a.H) break;
        const double yh = a.sy * y + a.oy;
        double yp[DS + 1];
        yp[0] = 1.0;
#pragma unroll
        for (int q = 1; q <= DS; ++q) yp[q] = yp[q - 1] * yh;
        // spatial term m = t (t + 1) / 2 + j is xh^(t - j) yh^j
        double v = 0.0;
        int m = 0;
#pragma unroll
        for (int t = 0; t <= DS; ++t)
#pragma unroll
            for (int j = 0; j <= t; ++j, ++m)
                v = fma(xp[t - j] * yp[j], fma((double)a.ped, gam_s[m], tot[o][m]), v);
        const size_t idx = (size_t)y * a.W + x;
        a.out[idx] = (float)(a.I ? v - (double)iv[o] : v);
    }
}

template <int H, bool DFB>
static void launch_direct_h(const DirectArgs& a, dim3 grid, hipStream_t s) {
    switch (a.d_s) {
        case 0: hipLaunchKernelGGL((contract_direct_kernel<H, 0, DFB>), grid, dim3(DR_NT), 0, s, a); break;
        case 1: hipLaunchKernelGGL((contract_direct_kernel<H, 1, DFB>), grid, dim3(DR_NT), 0, s, a); break;
        default: hipLaunchKernelGGL((contract_direct_kernel<H, 2, DFB>), grid, dim3(DR_NT), 0, s, a); break;
    }
}

bool direct_supported(int h, int d_s) { return h >= 1 && h <= kDirectMaxHalfWidth && d_s <= 2; }

int launch_contract_direct(DirectArgs a, bool dfb, hipStream_t s) {
    if (!direct_supported(a.h, a.d_s) || a.M != (a.d_s + 1) * (a.d_s + 2) / 2)
        return fail(SVCONV_EUNSUPPORTED, "direct regrouped kernel needs 1 <= half-width <= 4 and spatial degree <= 2");
    a.tiles_x = (a.W + DR_TW - 1) / DR_TW;
    const int tiles = a.tiles_x * ((a.H + DR_TH - 1) / DR_TH);
    if (tiles == 0) return SVCONV_OK;
    const dim3 grid(tiles);
    switch (a.h) {
        case 1: dfb ? launch_direct_h<1, true>(a, grid, s) : launch_direct_h<1, false>(a, grid, s); break;
        case 2: dfb ? launch_direct_h<2, true>(a, grid, s) : launch_direct_h<2, false>(a, grid, s); break;
        case 3: dfb ? launch_direct_h<3, true>(a, grid, s) : launch_direct_h<3, false>(a, grid, s); break;
        default: dfb ? launch_direct_h<4, true>(a, grid, s) : launch_direct_h<4, false>(a, grid, s); break;
    }
    return hip_status(hipGetLastError(), "contract_direct_kernel");
}

}  // namespace svc
