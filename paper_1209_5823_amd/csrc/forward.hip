// Forward contraction of the spatially-varying convolution on gfx950.
//
// Every forward-shaped computation of the library is one "weighted
// multi-filter correlation":
//
//   out(p) = sum_f w_f(p) * T_f(p) - I(p),
//   T_f(p) = sum_{dv,du} F_f[dv][du] * X(p + (du - h, dv - h)),
//
// with w_f(p) = sum_m coef[f][m] P_m(p) (basis form, Eq. 2 - Eq. 3) or
// w_f(p) = P_f(p) (regrouped form and the adjoint in R).  The T_f of a tile
// of output pixels are a dense product (filters x taps) . (taps x pixels) run
// on the matrix cores; the patch matrix is never stored: its columns are read
// straight out of an LDS copy of the input tile plus its halo.
#include <cstdlib>

#include "internal.hpp"

namespace svc {

typedef float f4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------- helpers --

// Workgroups are dispatched round-robin over the 8 XCDs.  Give each XCD a
// contiguous run of tiles so that neighbouring tiles (which share halo rows)
// meet in the same L2.
__device__ __forceinline__ int xcd_remap(int bid, int n) {
    const int x = bid & 7, t = bid >> 3;
    const int q = n >> 3, r = n & 7;
    return x * q + (x < r ? x : r) + t;
}

__device__ __forceinline__ double ipow_d(double x, int e) {
    double r = 1.0;
#pragma unroll
    for (int t = 0; t < kMaxSpatialDegree; ++t)
        if (t < e) r *= x;
    return r;
}

// Exponents (i, j) of spatial term m: t = 0..d, i = t..0, j = t - i.
__device__ __forceinline__ void term_exponents(int m, int& i, int& j) {
    int t = 0;
    while ((t + 1) * (t + 2) / 2 <= m) ++t;
    const int o = m - t * (t + 1) / 2;
    i = t - o;
    j = o;
}

// ------------------------------------------------------ FP32 geometry ----

constexpr int F32_TW = 64;   // output tile width: 4 waves x 16 columns
// LDS row pitch in floats for every kernel width: at least the widest tile
// row (64 + 2 kMaxHalfWidth samples) and 16 mod 64, so that the four rows a
// B-operand read spans fall on disjoint banks; a fixed pitch makes every row
// offset of the contraction an immediate.
constexpr int F32_PITCH = 144;
static_assert(F32_TW + 2 * kMaxHalfWidth <= F32_PITCH && F32_PITCH % 64 == 16, "FP32 LDS pitch");

// Output rows per tile (= 16-pixel blocks per wave): fewer rows for more
// filter blocks so that the float32 sub-chain and float64 total fit in 256
// registers (two waves per SIMD) without spilling.  The two-row packed form
// keeps the 8 rows of one block: 16 rows per tile measured slower.
constexpr int f32_tile_h(int nb) { return nb >= 3 ? 3 : nb >= 2 ? 4 : 8; }

// Two-row packing: with at most 8 filters, rows 8..15 of the 16-row A operand
// would be zeros.  They carry the same filters shifted down by one kernel row
// instead, so that the product over the input rows of output row y also yields
// output row y + 1 (the taps (dv, du) of row y + 1 see the input rows of taps
// (dv + 1, du) of row y).  Only every other output row then needs products.
bool f32_packed(int NF) { return NF <= 8; }

F32Geometry f32_geometry(int k, int nb) {
    F32Geometry g;
    g.k = k;
    g.n_rg = (k + 3) / 4;
    g.n_chunks = (g.n_rg * k + 3) / 4 * 4;   // padded to whole groups of 4 chunks
    g.nb = nb;
    g.tile_w = F32_TW;
    g.tile_h = f32_tile_h(nb);
    g.lds_rows = g.tile_h + 4 * g.n_rg - 1;
    g.lds_cols = g.tile_w + k - 1;
    g.lds_pitch = F32_PITCH;
    g.lds_bytes = (size_t)g.lds_rows * g.lds_pitch * 4 + (size_t)kMaxFilters * kMaxSpatialTerms * 4;
    return g;
}

size_t f32_fragment_floats(int k, int nb) {
    const F32Geometry g = f32_geometry(k, nb);
    return (size_t)g.n_chunks * nb * 64;
}

// A-operand fragments of v_mfma_f32_16x16x4_f32.  Chunk c = r * k + du holds
// the taps (dv = 4r + g, du), g = 0..3; lane l of block b carries filter
// 16 b + (l & 15) at tap g = l >> 4.  Packed (one block): lane l carries filter
// l & 7 at tap (dv - s, du) with s = (l >> 3) & 1, the shifted copy for the
// next output row.  Filters beyond NF and rows outside 0..k-1 are 0.
__global__ void frag_f32_kernel(const float* __restrict__ F, int NF, int k, int nb, int n_chunks,
                                int packed, float* __restrict__ frag) {
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long total = (long)n_chunks * nb * 64;
    if (idx >= total) return;
    const int lane = (int)(idx & 63);
    const int b = (int)((idx >> 6) % nb);
    const int c = (int)((idx >> 6) / nb);
    const int r = c / k, du = c - r * k;
    const int dv = 4 * r + (lane >> 4) - (packed ? (lane >> 3) & 1 : 0);
    const int f = packed ? (lane & 7) : 16 * b + (lane & 15);
    // chunks past the last row group (padding to a group of 4) carry zeros
    frag[idx] = (f < NF && dv >= 0 && dv < k) ? F[((size_t)f * k + dv) * k + du] : 0.f;
}

int build_f32_fragments(const float* F, int NF, int k, float* frag, hipStream_t s) {
    const int nb = (NF + 15) / 16;
    const F32Geometry g = f32_geometry(k, nb);
    const long total = (long)g.n_chunks * nb * 64;
    hipLaunchKernelGGL(frag_f32_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, F,
                       NF, k, nb, g.n_chunks, f32_packed(NF) ? 1 : 0, frag);
    return hip_status(hipGetLastError(), "frag_f32_kernel");
}

// ------------------------------------------------ FP32 contraction ----

template <int NB, int TH, bool REG, bool PACK>
__global__ __launch_bounds__(256, 2) void contract_f32_kernel(ContractArgs a,
                                                           const float* __restrict__ frag, int k,
                                                           int n_rg, int rows, int cols,
                                                           int tiles_x, int n_tiles) {
    static_assert(!PACK || (NB == 1 && TH % 2 == 0), "packed form: one filter block, row pairs");
    // products per chunk and filter block, and the tile-row step between them
    constexpr int RI = PACK ? TH / 2 : TH;
    constexpr int RS = PACK ? 2 : 1;
    extern __shared__ __align__(16) float smem[];
    float* tile = smem;
    constexpr int pitch = F32_PITCH;
    float* coef_s = smem + rows * pitch;

    const int tid = threadIdx.x;
    const int t = xcd_remap(blockIdx.x, n_tiles);
    const int X0 = (t % tiles_x) * F32_TW;
    const int Y0 = a.y_begin + (t / tiles_x) * TH;
    const int y_end = a.y_begin + a.n_rows;
    const int h = a.h;

    const bool want_d = (a.out != nullptr);   // false: only the T_f planes are written
    if (!REG && want_d)
        for (int q = tid; q < a.NF * a.M; q += 256) coef_s[q] = a.coef[q];

    // Stage X[Y0-h .. Y0-h+rows) x [X0-h .. X0-h+cols) minus the pedestal;
    // outside the image X is 0, so the staged value is -pedestal there.  A
    // lane covers columns c and c + 64 (cols <= 64 + 2 kMaxHalfWidth < 128)
    // of every fourth row; the loads of F32_SB rows are issued together from
    // clamped addresses and the masks apply when storing, so that a batch
    // waits for memory once.
    {
        constexpr int F32_SB = 4;
        int gxc[2];
        bool cin[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int c = (tid & 63) + 64 * q;
            const int gx = X0 - h + c;
            cin[q] = c < cols && gx >= 0 && gx < a.W;
            gxc[q] = gx < 0 ? 0 : (gx < a.W ? gx : a.W - 1);
        }
        for (int r0 = tid >> 6; r0 < rows; r0 += 4 * F32_SB) {
            float v[F32_SB][2];
#pragma unroll
            for (int sb = 0; sb < F32_SB; ++sb) {
                const int gy = Y0 - h + r0 + 4 * sb;
                const float* src = a.X + (size_t)(gy < 0 ? 0 : (gy < a.H ? gy : a.H - 1)) * a.W;
#pragma unroll
                for (int q = 0; q < 2; ++q) v[sb][q] = src[gxc[q]];
            }
#pragma unroll
            for (int sb = 0; sb < F32_SB; ++sb) {
                const int r = r0 + 4 * sb, gy = Y0 - h + r;
                const bool rin = gy >= 0 && gy < a.H;
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    const int c = (tid & 63) + 64 * q;
                    if (r < rows && c < cols) tile[r * pitch + c] = (rin && cin[q] ? v[sb][q] : 0.f) - a.ped;
                }
            }
        }
    }
    __syncthreads();

    const int lane = tid & 63, w = tid >> 6;
    const int g = lane >> 4, j = lane & 15;
    const int n_chunks = (n_rg * k + 3) / 4 * 4;

    // Lane (g, j) of product i ends with T_f at pixel column j of output row
    // Y0 + RS i + yo for f = 16 b + fo + e, e = 0..3; lanes with g_lead sum
    // the filters of their row and write it.
    const int fo = PACK ? 4 * (g & 1) : 4 * g;
    const int yo = PACK ? (g >> 1) : 0;
    const bool g_lead = PACK ? ((g & 1) == 0) : (g == 0);

    // I at this lane's output pixels, loaded now so that its latency hides
    // behind the contraction; clamped addresses (X stands in when there is no
    // I), the values of pixels outside the band are never used
    float iv[RI];
    {
        const float* ip = (a.I != nullptr) ? a.I : a.X;
        const int x = X0 + 16 * w + j, xc = x < a.W ? x : a.W - 1;
#pragma unroll
        for (int i = 0; i < RI; ++i) {
            const int y = Y0 + RS * i + yo, yc = y < y_end ? y : y_end - 1;
            iv[i] = ip[(size_t)yc * a.W + xc];
        }
    }

    // T_f accumulates on the matrix cores in float32 over sub-chains of 4
    // chunks (16 taps), and every sub-chain (with up to two filter blocks, the
    // float32 sum of two) is added into a float64 total.  Long float32 chains
    // over all k^2 taps lose up to a few ulp of T at bright stars; short
    // chains keep the rounding of each partial sum small and the float64
    // total adds none.
    double tot[NB][RI][4];
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int i = 0; i < RI; ++i)
#pragma unroll
            for (int e = 0; e < 4; ++e) tot[b][i][e] = 0.0;

    // The A fragments of a group of 4 chunks go to one of two register sets
    // while the other set's group runs: the loop takes two groups per turn so
    // that no set is copied (a copy of a value still in flight waits for it).
    // With up to two filter blocks a scheduling barrier keeps each group's
    // loads ahead of the products of the group before it; with more, the
    // compiler keeps that order by itself and the barrier would cost spills.
    const float* fp = frag + lane;
    auto load_group = [&](float (&f)[4][NB], int c0) {
        const int cc = (c0 < n_chunks) ? c0 : n_chunks - 4;   // past the end: unused
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int b = 0; b < NB; ++b) f[u][b] = fp[(size_t)((cc + u) * NB + b) * 64];
    };
    const float* tb = tile + g * pitch + 16 * w + j;
    int r = 0, du = 0;       // row group and column of the chunk being issued
    auto run_group = [&](const float (&f)[4][NB], f4 (&acc)[NB][RI]) {
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int i = 0; i < RI; ++i) acc[b][i] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            // padded chunks past the last row group read row group n_rg - 1
            // (in the tile) with zero weights
            const float* rb = tb + 4 * (r < n_rg ? r : n_rg - 1) * pitch + du;
            float xb[RI];
#pragma unroll
            for (int i = 0; i < RI; ++i) xb[i] = rb[RS * i * pitch];
#pragma unroll
            for (int i = 0; i < RI; ++i)
#pragma unroll
                for (int b = 0; b < NB; ++b)
                    acc[b][i] = __builtin_amdgcn_mfma_f32_16x16x4f32(f[u][b], xb[i], acc[b][i], 0, 0, 0);
            if (++du == k) {
                du = 0;
                ++r;
            }
        }
    };
    auto add_total = [&](const f4 (&acc)[NB][RI]) {
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int i = 0; i < RI; ++i)
#pragma unroll
                for (int e = 0; e < 4; ++e) tot[b][i][e] += (double)acc[b][i][e];
    };
    // With one or two filter blocks the sub-chains of the two groups of a turn
    // are added in float32 (one more rounding per 32 taps) before their sum
    // goes into the float64 total: half the conversions and float64 adds.
    constexpr bool PAIR = NB <= 2;
    // (The loop body is one basic block: loads in a block of their own would
    // be sunk next to their first use.)
    float fA[4][NB], fB[4][NB];
    load_group(fA, 0);
    int c0 = 0;
    for (; c0 + 8 <= n_chunks; c0 += 8) {
        load_group(fB, c0 + 4);
        if (NB < 3) __builtin_amdgcn_sched_barrier(0);
        f4 accA[NB][RI];
        run_group(fA, accA);
        if (!PAIR) add_total(accA);
        load_group(fA, c0 + 8);
        if (NB < 3) __builtin_amdgcn_sched_barrier(0);
        f4 accB[NB][RI];
        run_group(fB, accB);
        if (PAIR) {
#pragma unroll
            for (int b = 0; b < NB; ++b)
#pragma unroll
                for (int i = 0; i < RI; ++i) accB[b][i] += accA[b][i];
        }
        add_total(accB);
    }
    if (c0 < n_chunks) {   // an odd number of groups
        f4 accA[NB][RI];
        run_group(fA, accA);
        add_total(accA);
    }

    // Epilogue in float64: out = sum_f w_f (T_f + ped * beta_f) - I.
    const int x = X0 + 16 * w + j;
    const double xh = a.sx * x + a.ox;
    double xp[kMaxSpatialDegree + 1];
    xp[0] = 1.0;
#pragma unroll
    for (int q = 1; q <= kMaxSpatialDegree; ++q) xp[q] = xp[q - 1] * xh;

    // Per-filter terms of this lane's accumulator entries, formed once per
    // tile: ped * beta_f (loaded together from clamped indices) and, in the
    // regrouped form, the x power of monomial f and the exponent of its y power.
    double pbf[NB][4], wxf[NB][4];
    int jyf[NB][4];
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int f = 16 * b + fo + e;
            pbf[b][e] = 0.0;
            wxf[b][e] = 0.0;
            jyf[b][e] = 0;
            if (REG && want_d) {
                int ii, jj;
                term_exponents(f < a.NF ? f : 0, ii, jj);
                wxf[b][e] = ipow_d(xh, ii);
                jyf[b][e] = jj;
            }
        }
    if (a.beta != nullptr) {
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int f = 16 * b + fo + e;
                pbf[b][e] = (double)a.ped * a.beta[f < a.NF ? f : a.NF - 1];
            }
    }

#pragma unroll
    for (int i = 0; i < RI; ++i) {
        const int y = Y0 + RS * i + yo;
        const double yh = a.sy * y + a.oy;
        double yp[kMaxSpatialDegree + 1];
        yp[0] = 1.0;
#pragma unroll
        for (int q = 1; q <= kMaxSpatialDegree; ++q) yp[q] = yp[q - 1] * yh;
        // yh^j for j <= 7 from its binary digits, without branches
        const double yh2 = yh * yh, yh4 = yh2 * yh2;
        double part = 0.0;
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int f = 16 * b + fo + e;
                if (f < a.NF) {
                    double wgt = 0.0;
                    if (!want_d) {
                    } else if (REG) {
                        const int jj = jyf[b][e];
                        wgt = wxf[b][e] * (((jj & 1) ? yh : 1.0) * ((jj & 2) ? yh2 : 1.0)) *
                              ((jj & 4) ? yh4 : 1.0);
                    } else {
                        const float* cf = coef_s + f * a.M;
                        int m = 0;
#pragma unroll
                        for (int tt = 0; tt <= kMaxSpatialDegree; ++tt) {
                            if (tt <= a.d_s) {
#pragma unroll
                                for (int ii = tt; ii >= 0; --ii) wgt += (double)cf[m + tt - ii] * (xp[ii] * yp[tt - ii]);
                            }
                            m += tt + 1;
                        }
                    }
                    const double pb = pbf[b][e];
                    part += wgt * (tot[b][i][e] + pb);
                    if (a.tout != nullptr && x < a.W && y < y_end)
                        a.tout[(size_t)f * a.n_rows * a.W + (size_t)(y - a.y_begin) * a.W + x] =
                            (float)(tot[b][i][e] + pb);
                }
            }
        part += __shfl_xor(part, 16);
        if (!PACK) part += __shfl_xor(part, 32);
        if (a.out != nullptr && g_lead && x < a.W && y < y_end)
            a.out[(size_t)y * a.W + x] = (float)(part - (a.I != nullptr ? (double)iv[i] : 0.0));
    }
}

template <int NB, bool REG, bool PACK = false>
static int launch_f32_t(const ContractArgs& a, const float* frag, hipStream_t s) {
    constexpr int TH = f32_tile_h(NB);
    const int k = 2 * a.h + 1;
    const F32Geometry g = f32_geometry(k, NB);
    const int tiles_x = (a.W + g.tile_w - 1) / g.tile_w;
    const int tiles_y = (a.n_rows + g.tile_h - 1) / g.tile_h;
    const int n_tiles = tiles_x * tiles_y;
    if (n_tiles == 0) return SVCONV_OK;
    if (g.lds_bytes > 64 * 1024) return fail(SVCONV_EUNSUPPORTED, "FP32 tile exceeds 64 KiB of LDS");
    hipLaunchKernelGGL((contract_f32_kernel<NB, TH, REG, PACK>), dim3(n_tiles), dim3(256),
                       g.lds_bytes, s, a, frag, k, g.n_rg, g.lds_rows, g.lds_cols,
                       tiles_x, n_tiles);
    return hip_status(hipGetLastError(), "contract_f32_kernel");
}

int launch_contract_f32(const ContractArgs& a, const float* frag, int nb, hipStream_t s) {
    const bool reg = (a.coef == nullptr);
    if (nb == 1 && f32_packed(a.NF))
        return reg ? launch_f32_t<1, true, true>(a, frag, s)
                   : launch_f32_t<1, false, true>(a, frag, s);
    switch (nb) {
        case 1: return reg ? launch_f32_t<1, true>(a, frag, s) : launch_f32_t<1, false>(a, frag, s);
        case 2: return reg ? launch_f32_t<2, true>(a, frag, s) : launch_f32_t<2, false>(a, frag, s);
        case 3: return reg ? fail(SVCONV_EUNSUPPORTED, "regrouped form needs M <= 32")
                           : launch_f32_t<3, false>(a, frag, s);
        case 4: return reg ? fail(SVCONV_EUNSUPPORTED, "regrouped form needs M <= 32")
                           : launch_f32_t<4, false>(a, frag, s);
        default: return fail(SVCONV_EUNSUPPORTED, "more than 64 filters");
    }
}

// -------------------------------------------- per-call filter builders ----

// Regrouped filters Kt_m = sum_n a[n][m] F_n (float64 accumulation) and
// their sums beta_m = sum_n a[n][m] beta_n.
__global__ void regroup_kernel(const double* __restrict__ F64, const double* __restrict__ beta,
                               const float* __restrict__ a, int N, int M, int kk,
                               float* __restrict__ Ft, double* __restrict__ betaT) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < M * kk) {
        const int m = idx / kk, q = idx - m * kk;
        double s = 0.0;
        for (int n = 0; n < N; ++n) s += (double)a[n * M + m] * F64[(size_t)n * kk + q];
        Ft[idx] = (float)s;
    } else if (idx < M * kk + M) {
        const int m = idx - M * kk;
        double s = 0.0;
        for (int n = 0; n < N; ++n) s += (double)a[n * M + m] * beta[n];
        betaT[m] = s;
    }
}

int regroup_filters(const double* F64, const double* beta, const float* a, int N, int M, int k,
                    float* Ft, double* betaT, hipStream_t s) {
    const int total = M * k * k + M;
    hipLaunchKernelGGL(regroup_kernel, dim3((total + 255) / 256), dim3(256), 0, s, F64, beta, a, N,
                       M, k * k, Ft, betaT);
    return hip_status(hipGetLastError(), "regroup_kernel");
}

// Filters of the adjoint in R.  With Kt_m[u][v] = sum_n a[n][m] B_n[u][v],
//   dL/dR(q) = sum_{u,v} G(q + (u,v)) sum_m P_m(q + (u,v)) Kt_m[u][v],
// and P_m(q + (u,v)) expands binomially around q because xh(q + u) =
// xh(q) + u sx:  P_(i,j)(q+(u,v)) = sum_{i'<=i, j'<=j} C(i,i') C(j,j')
// (u sx)^(i-i') (v sy)^(j-j') P_(i',j')(q).  Hence
//   dL/dR(q) = sum_m' P_m'(q) sum_{u,v} H_m'[u][v] G(q + (u,v))
// with H_(i',j') = sum_{i>=i', j>=j'} C(i,i') C(j,j') (u sx)^(i-i') (v sy)^(j-j') Kt_(i,j):
// a correlation of G with M filters weighted by P_m'(q), i.e. the same
// contraction as the regrouped forward.  In correlation orientation
// F'_m'[dv][du] = H_m'[u = du - h][v = dv - h].  The float64 basis table holds
// F_n[dv][du] = B_n[2h - dv][2h - du], so B_n[u][v] (row v+h, column u+h)
// = F_n[h - v][h - u].
__global__ void adjoint_filter_kernel(const double* __restrict__ F64, const float* __restrict__ a,
                                      int N, int M, int k, double sx, double sy,
                                      float* __restrict__ Ft) {
    const int kk = k * k;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= M * kk) return;
    const int mp = idx / kk, q = idx - mp * kk;
    const int dv = q / k, du = q - dv * k;
    const int h = k / 2;
    const int u = du - h, v = dv - h;
    const int fq = (h - v) * k + (h - u);  // F_n index holding B_n[u][v]
    int ip, jp;
    term_exponents(mp, ip, jp);
    double acc = 0.0;
    for (int m = 0; m < M; ++m) {
        int i, jj;
        term_exponents(m, i, jj);
        if (i < ip || jj < jp) continue;
        double kt = 0.0;
        for (int n = 0; n < N; ++n) kt += (double)a[n * M + m] * F64[(size_t)n * kk + fq];
        // binomials C(i, ip) C(jj, jp)
        double ci = 1.0, cj = 1.0;
        for (int t = 1; t <= ip; ++t) ci = ci * (i - ip + t) / t;
        for (int t = 1; t <= jp; ++t) cj = cj * (jj - jp + t) / t;
        double px = 1.0, py = 1.0;
        for (int t = 0; t < i - ip; ++t) px *= u * sx;
        for (int t = 0; t < jj - jp; ++t) py *= v * sy;
        acc += ci * cj * px * py * kt;
    }
    Ft[idx] = (float)acc;
}

int adjoint_filters(const double* F64, const float* a, int N, int M, int d_s, int k, double sx,
                    double sy, float* Ft, hipStream_t s) {
    (void)d_s;
    const int total = M * k * k;
    hipLaunchKernelGGL(adjoint_filter_kernel, dim3((total + 255) / 256), dim3(256), 0, s, F64, a,
                       N, M, k, sx, sy, Ft);
    return hip_status(hipGetLastError(), "adjoint_filter_kernel");
}

}  // namespace svc
