// Regrouped separable form of the Gaussian-basis contraction on the matrix
// cores.
//
// With separable bases B_n(u,v) = f_i(u) f_j(v) (the row factor i and the
// column factor j of one Gaussian family) and constant weights a[n][m], the
// contraction of Eq. 1 - Eq. 3 regroups as
//   sum_n c_n(x,y) T_n(x,y) = sum_m P_m(x,y) Z_m(x,y),
//   Z_m = sum_n a[n][m] T_n = sum_r g_{r,m} (x)_y U_r,   U_r = f_r (x)_x R,
//   g_{r,m} = sum_j a[n(r,j)][m] f_j,
// because P_m depends only on the output pixel: one row pass per row factor
// r (all families together), then one column pass per row factor and
// spatial term with the per-call column filters g_{r,m}, accumulated over r.
// The coefficient weighting is folded into the column taps, so nothing but
// matrix-core products runs per basis.
//
// Both one-dimensional passes are banded Toeplitz products on
// v_mfma_f32_16x16x32_{f16,bf16}, laid out so that 28 of the 32 reduction
// entries are used for h <= 12 (8 outputs need 8 + 2h samples):
//   row pass:    A = 16 staged rows x 32 samples, B = taps of TWO row factors
//                x 8 output columns (n = 8 f + c);
//   column pass: A = taps of TWO spatial terms x 8 output rows (m = 8 s + y),
//                B = 32 row-response rows x 16 columns.
// The row responses never leave the registers: a lane of the row pass holds
// rows 4 g + e of one column (the accumulator layout), the column pass needs
// eight reduction entries per lane, and since a product sums over its whole
// reduction in any order, the K index of the column taps is permuted to the
// rows the lane already holds (two 16-row blocks: rows 4 g + e and
// 16 + 4 g + e; windows that start 8 rows into a block take the next block in
// lane groups 0 and 1).  The two factors of a row-pass product sit in lanes
// 0..7 and 8..15 of each DPP row; one DPP row rotation by 8 with a bank mask
// moves them into the 16-column layout of each factor.  The row-pass data
// window of the second 8-column group likewise reuses the loads of the first:
// its K index takes samples 8..31 from lane groups 1..3 and 32..39 from an
// extra load in lane group 0.
//
// Precision: 16-bit inputs, float32 accumulation, hi + lo splits of the
// data R - s (scaled by 1/4 in fp16), of the row responses and of both tap
// tables (Fh xh + Fh xl + Fl xh).  Each spatial term's column taps are scaled
// by a power of two (largest |tap| in [1, 2)), undone in the epilogue; the
// pedestal restore s sum_m gamma_m P_m and the subtraction of I in float32
// (sum_m P_m Z_m - I first, which is exact where both are large).
//
// Workgroup: 4 waves; output tile 64 x 64; wave w owns the 16-column strip
// w and every row of the tile.  LDS holds the staged tile (hi / lo rows
// [96][88]) and, per wave, the second factor's row responses while the
// first one's column passes run (written and read by the same lanes, so no
// barrier).  Workgroups are persistent, two per compute unit (the chip's
// 2048 tiles fall evenly on 512 workgroups); the only barriers are the ends
// of staging.
#include "internal.hpp"
#include "sep_fold.hpp"

namespace svc {

typedef float sz_f4 __attribute__((ext_vector_type(4)));
typedef _Float16 sz_h8 __attribute__((ext_vector_type(8)));
typedef __bf16 sz_b8 __attribute__((ext_vector_type(8)));

constexpr int SZ_NW = 4;                  // waves per workgroup (16-column strips)
constexpr int SZ_NT = 64 * SZ_NW;
constexpr int SZ_TW = 16 * SZ_NW;         // tile width
constexpr int SZ_OB = 8;                  // 8-row output blocks of a strip (even)
constexpr int SZ_MINW = 2;                // waves per SIMD the registers allow
constexpr int SZ_TH = 8 * SZ_OB;          // tile height
constexpr int SZ_RB = SZ_OB / 2 + 2;      // 16-row blocks of row responses (16 SZ_RB >= SZ_TH + 2h for h <= 12)
constexpr int SZ_XR = 16 * SZ_RB;         // staged rows
constexpr int SZ_XC = SZ_TW + 24;         // staged columns the windows reach (88)
constexpr int SZ_P = SZ_XC;               // pitch in 16-bit elements: 11 x 16 B (odd)
constexpr int SZ_FRAG = 2 * 2 * 64 * 8;   // one table entry: [2 (cg or phase)][hi/lo][lane][8]
constexpr size_t SZ_XLDS = (size_t)2 * SZ_XR * SZ_P * sizeof(uint16_t);     // staged tile
constexpr size_t SZ_LDS = SZ_XLDS + (size_t)SZ_NW * SZ_RB * 64 * 16;         // + per-wave factor-B rows

__device__ __forceinline__ uint32_t sz_f2h(float x) { return (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)x); }
__device__ __forceinline__ float sz_h2f(uint32_t b) { return (float)__builtin_bit_cast(_Float16, (uint16_t)b); }
__device__ __forceinline__ uint32_t sz_f2bf(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return u >> 16;
}
__device__ __forceinline__ float sz_bf2f(uint32_t b) { return __uint_as_float(b << 16); }

// A float64 table value split into rounded 16-bit hi and lo parts.
template <bool FP16>
__device__ __forceinline__ void sz_split_tap(double v, uint16_t& hi, uint16_t& lo) {
    if (FP16) {
        const uint32_t h = sz_f2h((float)v);
        hi = (uint16_t)h;
        lo = (uint16_t)sz_f2h((float)(v - (double)sz_h2f(h)));
    } else {
        const uint32_t h = sz_f2bf((float)v);
        hi = (uint16_t)h;
        lo = (uint16_t)sz_f2bf((float)(v - (double)sz_bf2f(h)));
    }
}

// lo parts of two float32 values whose fp16 hi parts are packed in hv:
// (x - hi) formed exactly and rounded to fp16 (nearest even) in one
// mixed-precision FMA per value, written into the low and the high half.
__device__ __forceinline__ uint32_t sz_lo2_f16(uint32_t hv, float x0, float x1) {
    uint32_t lo;
    asm("v_fma_mixlo_f16 %0, %1, -1.0, %2 op_sel_hi:[1,0,0]" : "=v"(lo) : "v"(hv), "v"(x0));
    asm("v_fma_mixhi_f16 %0, %1, -1.0, %2 op_sel:[1,0,0] op_sel_hi:[1,0,0]" : "+v"(lo) : "v"(hv), "v"(x1));
    return lo;
}

// Two float32 values split into packed hi and lo parts.  fp16: hi by the
// packed truncating conversion, lo the remainder x - hi (exact in float32)
// rounded to nearest even; bf16: both rounded to nearest even.
template <bool FP16>
__device__ __forceinline__ void sz_split2(float x0, float x1, uint32_t& hi2, uint32_t& lo2) {
    if (FP16) {
        hi2 = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_pkrtz(x0, x1));
        lo2 = sz_lo2_f16(hi2, x0, x1);
    } else {
        const uint32_t h0 = sz_f2bf(x0), h1 = sz_f2bf(x1);
        const uint32_t l0 = sz_f2bf(x0 - sz_bf2f(h0)), l1 = sz_f2bf(x1 - sz_bf2f(h1));
        hi2 = h0 | (h1 << 16);
        lo2 = l0 | (l1 << 16);
    }
}

template <bool FP16>
__device__ __forceinline__ sz_f4 sz_mfma(const uint4& a, const uint4& b, sz_f4 c) {
    if constexpr (FP16) {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(sz_h8, a), __builtin_bit_cast(sz_h8, b), c,
                                                      0, 0, 0);
    } else {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(sz_b8, a), __builtin_bit_cast(sz_b8, b), c,
                                                       0, 0, 0);
    }
}

// Sample offset (within the 40-sample data window of a strip) that reduction
// entry (lane group g, element t) of the row pass stands for: the first
// 8-column group reads samples 8 g + t, the second reuses them in lane groups
// 1..3 and reads samples 32 + t in lane group 0.
__host__ __device__ __forceinline__ int sz_row_sample(int cg, int g, int t) {
    return (cg == 1 && g == 0) ? 32 + t : 8 * g + t;
}

// Row-response row (relative to the first output row of an 8-row block) that
// reduction entry (g, t) of the column pass stands for; phase 0 blocks start
// on a 16-row block boundary (entries t < 4 from block b, t >= 4 from block
// b + 1), phase 1 blocks 8 rows into one (t < 4 from block b + 1 in every
// lane group, t >= 4 from block b + 2 in lane groups 0, 1 and from block b
// in groups 2, 3), so that only half of a phase 1 operand is chosen per lane.
__host__ __device__ __forceinline__ int sz_col_row(int ph, int g, int t) {
    if (!ph) return (t < 4 ? 0 : 16) + 4 * g + (t & 3);
    return (t < 4 ? 8 : (g < 2 ? 24 : -8)) + 4 * g + (t & 3);
}

// Row-pass tap tables, fp16 then bf16 (or only precision p0 when np = 1):
// rtab[p - p0][pp][cg][hl][lane][t] = split(f_r(8 cg + c + 2h - s)),
// r = 2 pp + (n >= 8), c = n mod 8, n = lane mod 16,
// s = sz_row_sample(cg, lane / 16, t); zero outside [0, 2h] and for r >= R.
__global__ void sepz_rtab_kernel(const double* __restrict__ f1d, const int* __restrict__ rinfo, int R, int h,
                                 int p0, int np, uint16_t* __restrict__ rtab) {
    const int n_pairs = (R + 1) / 2;
    const long total = (long)np * n_pairs * 2 * 64 * 8;      // [p][pp][cg][lane][t]
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int t = (int)(idx & 7), lane = (int)((idx >> 3) & 63), cg = (int)((idx >> 9) & 1);
    const long rest = idx >> 10;
    const int pp = (int)(rest % n_pairs), pq = (int)(rest / n_pairs);
    const int n = lane & 15, g = lane >> 4, r = 2 * pp + (n >> 3), c = n & 7;
    const int k = 2 * h + 1;
    const int u = 8 * cg + c + 2 * h - sz_row_sample(cg, g, t);
    double v = 0.0;
    if (r < R && u >= 0 && u < k) v = f1d[((size_t)rinfo[2 * r] * kSepMaxFactors + rinfo[2 * r + 1]) * k + u];
    uint16_t hi, lo;
    if (p0 + pq == 0) sz_split_tap<true>(v, hi, lo);
    else sz_split_tap<false>(v, hi, lo);
    uint16_t* dst = rtab + ((size_t)pq * n_pairs + pp) * SZ_FRAG;
    dst[((cg * 2 + 0) * 64 + lane) * 8 + t] = hi;
    dst[((cg * 2 + 1) * 64 + lane) * 8 + t] = lo;
}

size_t sepz_rtab_entries(int R) { return 2 * (size_t)((R + 1) / 2) * SZ_FRAG; }
size_t sepz_ztab_entries(int R) { return (size_t)R * 3 * SZ_FRAG; }

int build_sepz_rtab(const double* f1d, const int* rinfo, int R, int h, uint16_t* rtab, hipStream_t s, int only) {
    const int p0 = only < 0 ? 0 : only, np = only < 0 ? 2 : 1;
    const long total = (long)np * ((R + 1) / 2) * 2 * 64 * 8;
    hipLaunchKernelGGL(sepz_rtab_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, f1d, rinfo, R, h,
                       p0, np, rtab);
    return hip_status(hipGetLastError(), "sepz_rtab_kernel");
}

// Value of the regrouped column filter g_{r,m} at tap u (float64):
// sum_j a[n(r,j)][m] f_j(u) over the column factors j of row factor r's
// family (the family's factors are row factors r - i .. r - i + degree), from
// the block's copies of a and of the factors; i is r's index in its family,
// deg and base the family's degree and first basis.
__device__ __forceinline__ double sz_gval(const float* as, const double* fcs, int i, int deg, int base, int M, int k,
                                          int r, int m, int u) {
    double s = 0.0;
    for (int j = 0; j + i <= deg; ++j) {
        const int tt = i + j;
        const int n = base + tt * (tt + 1) / 2 + j;
        s = fma((double)as[n * M + m], fcs[(r - i + j) * k + u], s);
    }
    return s;
}

constexpr int kSzPrepMaxRows = 64;   // row factors (N <= 64)

// Per-call tables: block (r, mp) writes the column-pass fragments of row
// factor r and spatial terms 2 mp, 2 mp + 1 (both phases, hi and lo):
// ztab[r][mp][ph][hl][lane][t] = split(S_m g_{r,m}(y + 2h - rho)), m = 2 mp +
// (lane mod 16) / 8, y = lane mod 8, rho = sz_col_row(ph, lane / 16, t), zero
// outside [0, 2h] and for m >= M; S_m is the power of two that puts the
// largest |g_{., m}| in [1, 2).  Blocks of r = 0 also write zinv[m] =
// 1 / (S_m xscale), and block (0, 0) the padded pedestal sums
// gam[m] = sum_n a[n][m] beta_n.  a, beta and the factors are first copied
// into LDS (every load of a phase in flight together), so the sums read no
// global memory; the maxima reduce across each wave by shuffles.
template <bool FP16>
__global__ __launch_bounds__(256) void sepz_prep_kernel(const float* __restrict__ a, const double* __restrict__ f1d,
                                                        const int* __restrict__ rinfo, const int* __restrict__ fam,
                                                        const double* __restrict__ beta, int R, int N, int M, int h,
                                                        float xscale, uint16_t* __restrict__ ztab,
                                                        float* __restrict__ zinv, double* __restrict__ gam) {
    constexpr int KMAX = 2 * kSepZMaxHalfWidth + 1;
    __shared__ double red[2][4];
    __shared__ double scale[2];
    __shared__ double fcs[kSzPrepMaxRows * KMAX];
    __shared__ double bt[kMaxFilters];
    __shared__ float as[kMaxFilters * 6];
    __shared__ int ri[2 * kSzPrepMaxRows];
    __shared__ int rfam[2 * kSzPrepMaxRows];   // per row factor: family degree, first basis
    const int r = blockIdx.x, mp = blockIdx.y, tid = threadIdx.x;
    const int k = 2 * h + 1;
    // a, beta and the row factors' (family, index) pairs; clamped addresses,
    // so that no load is conditional
    constexpr int NA = (kMaxFilters * 6 + 255) / 256;
    {
        float av[NA];
#pragma unroll
        for (int i = 0; i < NA; ++i) av[i] = a[min(tid + 256 * i, N * M - 1)];
        const int rv = rinfo[min(tid, 2 * R - 1)];
        const double bv = beta[min(tid, N - 1)];
#pragma unroll
        for (int i = 0; i < NA; ++i)
            if (tid + 256 * i < N * M) as[tid + 256 * i] = av[i];
        if (tid < 2 * R) ri[tid] = rv;
        if (tid < N) bt[tid] = bv;
    }
    __syncthreads();
    constexpr int NF = (kSzPrepMaxRows * KMAX + 255) / 256;
    {
        double fv[NF];
#pragma unroll
        for (int i = 0; i < NF; ++i) {
            const int q = min(tid + 256 * i, R * k - 1);
            const int rr = q / k, u = q - rr * k;
            fv[i] = f1d[((size_t)ri[2 * rr] * kSepMaxFactors + ri[2 * rr + 1]) * k + u];
        }
        const int fr = min(tid, R - 1);
        const int fd = fam[2 * ri[2 * fr]], fb = fam[2 * ri[2 * fr] + 1];
#pragma unroll
        for (int i = 0; i < NF; ++i)
            if (tid + 256 * i < R * k) fcs[tid + 256 * i] = fv[i];
        if (tid < R) {
            rfam[2 * tid] = fd;
            rfam[2 * tid + 1] = fb;
        }
    }
    __syncthreads();
    // largest |g_{r', m}| over every row factor and tap, for m = 2 mp + s
    double mx[2] = {0.0, 0.0};
    for (int q = tid; q < R * k; q += 256) {
        const int rr = q / k, u = q - rr * k;
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const int m = 2 * mp + s;
            if (m < M)
                mx[s] = fmax(mx[s], fabs(sz_gval(as, fcs, ri[2 * rr + 1], rfam[2 * rr], rfam[2 * rr + 1], M, k, rr, m, u)));
        }
    }
#pragma unroll
    for (int s = 0; s < 2; ++s) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) mx[s] = fmax(mx[s], __shfl_xor(mx[s], off));
        if ((tid & 63) == 0) red[s][tid >> 6] = mx[s];
    }
    __syncthreads();
    if (tid < 2) {
        const double v = fmax(fmax(red[tid][0], red[tid][1]), fmax(red[tid][2], red[tid][3]));
        double sc = 1.0;
        if (v > 0.0) {
            int e;
            (void)frexp(v, &e);          // v = f 2^e, f in [0.5, 1)
            sc = ldexp(1.0, 1 - e);      // v sc in [1, 2)
        }
        scale[tid] = sc;
        const int m = 2 * mp + tid;
        if (r == 0 && m < M) zinv[m] = (float)(1.0 / (sc * (double)xscale));
    }
    if (r == 0 && mp == 0 && tid < kSepCoefPad) {
        double s = 0.0;
        if (tid < M)
            for (int n = 0; n < N; ++n) s = fma((double)as[n * M + tid], bt[n], s);
        gam[tid] = s;
    }
    __syncthreads();
    uint16_t* dst = ztab + ((size_t)r * 3 + mp) * SZ_FRAG;
    for (int q = tid; q < 2 * 64 * 8; q += 256) {
        const int t = q & 7, lane = (q >> 3) & 63, ph = q >> 9;
        const int s = (lane & 15) >> 3, y = lane & 7, g = lane >> 4;
        const int m = 2 * mp + s;
        const int u = y + 2 * h - sz_col_row(ph, g, t);
        double v = 0.0;
        if (m < M && u >= 0 && u < k) v = scale[s] * sz_gval(as, fcs, ri[2 * r + 1], rfam[2 * r], rfam[2 * r + 1], M, k, r, m, u);
        uint16_t hi, lo;
        sz_split_tap<FP16>(v, hi, lo);
        dst[((ph * 2 + 0) * 64 + lane) * 8 + t] = hi;
        dst[((ph * 2 + 1) * 64 + lane) * 8 + t] = lo;
    }
}

int launch_sepz_prep(const SepZArgs& z, const float* a, const double* f1d, const int* fam, const double* beta, int N,
                     bool fp16, hipStream_t s) {
    if (z.R > kSzPrepMaxRows || N > kMaxFilters || z.M > 6 || z.h > kSepZMaxHalfWidth)
        return fail(SVCONV_EUNSUPPORTED, "regrouped separable tables: at most 64 row factors, 64 bases, 6 terms");
    const int MP = (z.M + 1) / 2;
    const float xscale = fp16 ? 0.25f : 1.f;
    if (fp16)
        hipLaunchKernelGGL(sepz_prep_kernel<true>, dim3(z.R, MP), dim3(256), 0, s, a, f1d, z.rinfo, fam, beta, z.R, N,
                           z.M, z.h, xscale, const_cast<uint16_t*>(z.ztab), const_cast<float*>(z.zinv),
                           const_cast<double*>(z.gam));
    else
        hipLaunchKernelGGL(sepz_prep_kernel<false>, dim3(z.R, MP), dim3(256), 0, s, a, f1d, z.rinfo, fam, beta, z.R, N,
                           z.M, z.h, xscale, const_cast<uint16_t*>(z.ztab), const_cast<float*>(z.zinv),
                           const_cast<double*>(z.gam));
    return hip_status(hipGetLastError(), "sepz_prep_kernel");
}

// 16 bytes of LDS through an LDS-space pointer.
typedef const __attribute__((address_space(3))) uint16_t* lds_u16;
typedef unsigned int sz_u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ uint4 sz_lds16(lds_u16 p) {
    const sz_u32x4 v = *(const __attribute__((address_space(3))) sz_u32x4*)p;
    return make_uint4(v[0], v[1], v[2], v[3]);
}

// DPP row rotation by 8 lanes written only into the banks of bank_mask (the
// other lanes keep `old`).
template <int BANKS>
__device__ __forceinline__ uint32_t sz_ror8(uint32_t old, uint32_t src) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)src, 0x128, 0xf, BANKS, false);
}

// lo in lanes 0..31 (DPP rows 0 and 1), hi in lanes 32..63: a DPP move with
// the identity permutation and a row mask, so the choice stays a per-lane
// register move.
__device__ __forceinline__ uint32_t sz_sel_low(uint32_t lo, uint32_t hi) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)hi, (int)lo, 0xe4, 0x3, 0xf, false);
}

// One table entry (a row-pass pair or a column-pass spatial-term pair) for
// this lane: [cg or phase][hi/lo], 16 bytes each.
__device__ __forceinline__ void sz_load_tab(const uint16_t* __restrict__ tab, int lane, uint4 (&t)[2][2]) {
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int hl = 0; hl < 2; ++hl)
            t[c][hl] = *reinterpret_cast<const uint4*>(tab + ((c * 2 + hl) * 64 + lane) * 8);
    // keep the loads where they are issued: the scheduler would otherwise sink
    // them next to their use and expose the L2 latency
    __builtin_amdgcn_sched_barrier(0);
}

// Phase 1 column windows of one row factor, formed once for every spatial
// term: block b + 1, then block b + 2 (lane groups 0, 1) or block b (groups
// 2, 3).
__device__ __forceinline__ void sz_phase1_windows(const uint32_t (&Uh)[2 * SZ_RB], const uint32_t (&Ul)[2 * SZ_RB],
                                                  uint4 (&w1h)[SZ_OB / 2], uint4 (&w1l)[SZ_OB / 2]) {
#pragma unroll
    for (int b = 0; b < SZ_OB / 2; ++b) {
        w1h[b] = make_uint4(Uh[2 * b + 2], Uh[2 * b + 3], sz_sel_low(Uh[2 * b + 4], Uh[2 * b]),
                            sz_sel_low(Uh[2 * b + 5], Uh[2 * b + 1]));
        w1l[b] = make_uint4(Ul[2 * b + 2], Ul[2 * b + 3], sz_sel_low(Ul[2 * b + 4], Ul[2 * b]),
                            sz_sel_low(Ul[2 * b + 5], Ul[2 * b + 1]));
    }
}

// Column passes of one row factor r for spatial terms 2 mp, 2 mp + 1:
// Z[s][ob] += g_{r, 2 mp + s} (x)_y U_r for the output blocks of 8 rows
// (ob = 2 b: rows 16 b.., phase 0, window blocks b, b + 1; ob = 2 b + 1:
// rows 16 b + 8.., phase 1, window block b + 1, then block b + 2 in lane
// groups 0, 1 or block b in groups 2, 3).  Uh / Ul: the lane's row responses,
// two packed registers per 16-row block; za: the fragments [phase][hi/lo].
template <bool FP16, int NT>
__device__ __forceinline__ void sz_colpass(sz_f4 (&Z)[SZ_OB], const uint32_t (&Uh)[2 * SZ_RB],
                                           const uint32_t (&Ul)[2 * SZ_RB], const uint4 (&W1h)[SZ_OB / 2],
                                           const uint4 (&W1l)[SZ_OB / 2], const uint4 (&za)[2][2]) {
#pragma unroll
    for (int b = 0; b < SZ_OB / 2; ++b) {
        const uint4 w0h = make_uint4(Uh[2 * b], Uh[2 * b + 1], Uh[2 * b + 2], Uh[2 * b + 3]);
        const uint4 w0l = make_uint4(Ul[2 * b], Ul[2 * b + 1], Ul[2 * b + 2], Ul[2 * b + 3]);
        const uint4 w1h = W1h[b], w1l = W1l[b];
        Z[2 * b] = sz_mfma<FP16>(za[0][0], w0h, Z[2 * b]);
        Z[2 * b + 1] = sz_mfma<FP16>(za[1][0], w1h, Z[2 * b + 1]);
        if (NT >= 2) {
            Z[2 * b] = sz_mfma<FP16>(za[0][0], w0l, Z[2 * b]);
            Z[2 * b + 1] = sz_mfma<FP16>(za[1][0], w1l, Z[2 * b + 1]);
        }
        if (NT >= 3) {
            Z[2 * b] = sz_mfma<FP16>(za[0][1], w0h, Z[2 * b]);
            Z[2 * b + 1] = sz_mfma<FP16>(za[1][1], w1h, Z[2 * b + 1]);
        }
    }
}

// Staging of one tile, row by row: wave w stages rows w, w + 4, ... of the
// [SZ_XR][SZ_XC] window, lane l < SZ_XC / 2 the columns 2 l, 2 l + 1.  The row
// is uniform across the wave, so a row's address is scalar work and a lane's
// column offset (clamped into the image) is formed once per tile; no load is
// conditional, so all of them are in flight together.  Samples outside the
// image or past the halo are masked when they are stored.
constexpr int SZ_SROWS = SZ_XR / SZ_NW;   // staged rows per wave

// The samples of tile t this lane stages.
__device__ __forceinline__ void sz_load_tile(const SepZArgs& a, int t, int w, int lane, float (&sv)[SZ_SROWS][2]) {
    const int h = a.h;
    const int X0 = (t % a.tiles_x) * SZ_TW, Y0 = a.y_begin + (t / a.tiles_x) * SZ_TH;
    // the per-lane offsets are formed anew for every tile rather than kept in
    // registers across the tile loop
    asm volatile("" : "+v"(lane));
    uint32_t xb[2];
#pragma unroll
    for (int e = 0; e < 2; ++e) xb[e] = 4u * (uint32_t)min(max(X0 - h + 2 * min(lane, SZ_XC / 2 - 1) + e, 0), a.W - 1);
#pragma unroll
    for (int k = 0; k < SZ_SROWS; ++k) {
        const int gy = Y0 - h + w + SZ_NW * k;
        const char* row = reinterpret_cast<const char*>(a.X + (size_t)min(max(gy, 0), a.H - 1) * a.W);
#pragma unroll
        for (int e = 0; e < 2; ++e) sv[k][e] = *reinterpret_cast<const float*>(row + xb[e]);
    }
}

// The staged samples of tile t as (R - s) xscale split into hi / lo rows of the
// staged tile, with R = 0 outside the image; 0 past the halo (zero taps meet
// it).
template <bool FP16>
__device__ __forceinline__ void sz_store_tile(const SepZArgs& a, int t, int w, int lane,
                                              const float (&sv)[SZ_SROWS][2], uint16_t* xs) {
    if (lane >= SZ_XC / 2) return;
    const float xscale = FP16 ? 0.25f : 1.f;
    const float pscaled = a.ped * xscale;
    const int h = a.h;
    const int X0 = (t % a.tiles_x) * SZ_TW, Y0 = a.y_begin + (t / a.tiles_x) * SZ_TH;
    const int RA = SZ_TH + 2 * h, CA = SZ_TW + 2 * h;
    asm volatile("" : "+v"(lane));
    const int c = 2 * lane;
    bool cin[2], cimg[2];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        cin[e] = c + e < CA;
        cimg[e] = X0 - h + c + e >= 0 && X0 - h + c + e < a.W;
    }
    uint16_t* dst = xs + w * SZ_P + c;
#pragma unroll
    for (int k = 0; k < SZ_SROWS; ++k) {
        const int r = w + SZ_NW * k, gy = Y0 - h + r;
        const bool rin = r < RA, rimg = gy >= 0 && gy < a.H;
        float v[2];
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const float x = (rimg && cimg[e]) ? sv[k][e] : 0.f;
            v[e] = (rin && cin[e]) ? fmaf(x, xscale, -pscaled) : 0.f;
        }
        uint32_t hi2, lo2;
        sz_split2<FP16>(v[0], v[1], hi2, lo2);
        *reinterpret_cast<uint32_t*>(dst + SZ_NW * k * SZ_P) = hi2;
        *reinterpret_cast<uint32_t*>(dst + (SZ_XR + SZ_NW * k) * SZ_P) = lo2;
    }
}

// Persistent workgroups: workgroup b takes tiles b, b + G, b + 2G, ... (G =
// the grid) in the XCD-aware order; each wave requests its rows of the next
// tile once the current tile's epilogue is issued, and they are staged after
// the barrier that ends the current tile.
template <bool FP16, int NT, int MP>
__global__ __launch_bounds__(SZ_NT, SZ_MINW) void contract_sepz_kernel(SepZArgs a) {
    extern __shared__ uint4 sz_lds[];
    uint16_t* xs = reinterpret_cast<uint16_t*>(sz_lds);   // [2][SZ_XR][SZ_P]

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int g4 = lane >> 4, j16 = lane & 15;
    const int y_end = min(a.H, a.y_begin + a.n_rows);
    const int G = gridDim.x;
    // data offset of the second 8-column group's reduction entries in this lane
    const int off1 = g4 == 0 ? 32 : 8 * g4;
    // this lane's staged row in block 0 at the strip start, as an LDS-space
    // pointer so that the row loads stay LDS loads through the asm barrier below
    const lds_u16 xrow = (lds_u16)(xs + j16 * SZ_P + 16 * w);
    // this wave's area for the second factor's row responses: [SZ_RB][64 lanes] uint4
    uint4* ubw = sz_lds + SZ_XLDS / 16 + (size_t)w * SZ_RB * 64 + lane;
    const int n_pairs = (a.R + 1) / 2;

    // The tap tables are read one stage ahead: a stage is the row pass of a
    // pair of row factors or the column passes of one row factor for one pair
    // of spatial terms, and the next stage's entry is requested into `nxt`
    // before the current stage's products are issued (into registers of its
    // own), so its latency overlaps their execution (the tables are read from
    // L2).  The stage after a tile's last is the first one of the next tile.
    uint4 cur[2][2], nxt[2][2];
    sz_load_tab(a.rtab, lane, cur);

    // the per-call epilogue constants in LDS: zinv (zero for m >= M) and the
    // pedestal sums gamma_m as float32
    __shared__ float ep[16];
    if (tid < 16) ep[tid] = tid < 6 ? (tid < a.M ? a.zinv[tid] : 0.f) : (tid >= 8 && tid < 14 ? (float)a.gam[tid - 8] : 0.f);

    // the wave index as a scalar: the staged rows are uniform across a wave
    const int ws = __builtin_amdgcn_readfirstlane(w);
    int it = blockIdx.x;
    if (it < a.n_tiles) {
        const int t = sep_xcd_remap(it, a.n_tiles);
        float sv[SZ_SROWS][2];
        sz_load_tile(a, t, ws, lane, sv);
        sz_store_tile<FP16>(a, t, ws, lane, sv, xs);
    }
    __syncthreads();
    for (; it < a.n_tiles; it += G) {
        const int t = sep_xcd_remap(it, a.n_tiles);
        const int X0 = (t % a.tiles_x) * SZ_TW;
        const int Y0 = a.y_begin + (t / a.tiles_x) * SZ_TH;
        const bool more = it + G < a.n_tiles;
        const int tn = more ? sep_xcd_remap(it + G, a.n_tiles) : t;

        sz_f4 Z[MP][SZ_OB];
#pragma unroll
        for (int s = 0; s < MP; ++s)
#pragma unroll
            for (int b = 0; b < SZ_OB; ++b) Z[s][b] = sz_f4{0.f, 0.f, 0.f, 0.f};

        for (int pp = 0; pp < n_pairs; ++pp) {
            const bool has_b = 2 * pp + 1 < a.R;
            const uint16_t* ztA = a.ztab + (size_t)(2 * pp) * 3 * SZ_FRAG;
            const uint16_t* ztB = ztA + 3 * SZ_FRAG;
            // the entry after the last column stage of this pair: the next pair's
            // row-pass entry (the first one again after the last pair)
            const uint16_t* rnext = a.rtab + (size_t)(pp + 1 < n_pairs ? pp + 1 : 0) * SZ_FRAG;
            sz_load_tab(ztA, lane, nxt);
            // the staged rows are re-read for every pair rather than held in
            // registers across the loop (they would cost 48 registers per lane)
            lds_u16 xr = xrow;
            asm volatile("" : "+v"(xr));
            // ---- row pass: two row factors x two 8-column groups, SZ_RB row blocks.
            // The products of row block rb + 1 are issued before the split of
            // block rb, so the vector work of one block overlaps the matrix-core
            // work of the next.
            uint32_t UAh[2 * SZ_RB], UAl[2 * SZ_RB];
            sz_f4 acc[2][2];   // [rb parity][cg]
            auto issue = [&](int rb, sz_f4 (&ac)[2]) {
                // the second 8-column group reuses the samples of lane groups 1..3
                // and reads samples 32..39 in lane group 0
                const lds_u16 rp = xr + (16 * rb) * SZ_P;
                uint4 dh[2], dl[2];
                dh[0] = sz_lds16(rp + 8 * g4);
                dl[0] = sz_lds16(rp + SZ_XR * SZ_P + 8 * g4);
                dh[1] = sz_lds16(rp + off1);
                dl[1] = sz_lds16(rp + SZ_XR * SZ_P + off1);
#pragma unroll
                for (int cg = 0; cg < 2; ++cg) ac[cg] = sz_mfma<FP16>(dh[cg], cur[cg][0], sz_f4{0.f, 0.f, 0.f, 0.f});
                if (NT >= 2)
#pragma unroll
                    for (int cg = 0; cg < 2; ++cg) ac[cg] = sz_mfma<FP16>(dl[cg], cur[cg][0], ac[cg]);
                if (NT >= 3)
#pragma unroll
                    for (int cg = 0; cg < 2; ++cg) ac[cg] = sz_mfma<FP16>(dh[cg], cur[cg][1], ac[cg]);
            };
            // split, then move the two factors into the 16-column layout: factor A
            // holds lanes 0..7 of group 0 and (rotated) lanes 0..7 of group 1,
            // factor B (rotated) lanes 8..15 of group 0 and lanes 8..15 of group 1;
            // factor B waits in this wave's LDS area until its column pass
            auto split = [&](int rb, const sz_f4 (&ac)[2]) {
                uint32_t c0h[2], c0l[2], c1h[2], c1l[2];
                sz_split2<FP16>(ac[0][0], ac[0][1], c0h[0], c0l[0]);
                sz_split2<FP16>(ac[0][2], ac[0][3], c0h[1], c0l[1]);
                sz_split2<FP16>(ac[1][0], ac[1][1], c1h[0], c1l[0]);
                sz_split2<FP16>(ac[1][2], ac[1][3], c1h[1], c1l[1]);
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    UAh[2 * rb + e] = sz_ror8<0xc>(c0h[e], c1h[e]);
                    UAl[2 * rb + e] = sz_ror8<0xc>(c0l[e], c1l[e]);
                }
                ubw[rb * 64] = make_uint4(sz_ror8<0x3>(c1h[0], c0h[0]), sz_ror8<0x3>(c1h[1], c0h[1]),
                                          sz_ror8<0x3>(c1l[0], c0l[0]), sz_ror8<0x3>(c1l[1], c0l[1]));
            };
            // the row pass runs at raised wave priority: its vector work (splits,
            // row moves) then fills the issue cycles that the other wave's
            // column passes leave between their matrix-core products
            __builtin_amdgcn_s_setprio(1);
            issue(0, acc[0]);
#pragma unroll
            for (int rb = 1; rb < SZ_RB; ++rb) {
                issue(rb, acc[rb & 1]);
                split(rb - 1, acc[(rb - 1) & 1]);
            }
            split(SZ_RB - 1, acc[(SZ_RB - 1) & 1]);
            __builtin_amdgcn_s_setprio(0);

            // ---- column passes: Z[s][ob] += g_{r, 2 mp + s} (x)_y U_r for both factors
            {
                uint4 w1h[SZ_OB / 2], w1l[SZ_OB / 2];
                sz_phase1_windows(UAh, UAl, w1h, w1l);
#pragma unroll
                for (int mp = 0; mp < MP; ++mp) {
#pragma unroll
                    for (int c = 0; c < 2; ++c)
#pragma unroll
                        for (int hl = 0; hl < 2; ++hl) cur[c][hl] = nxt[c][hl];
                    sz_load_tab(mp + 1 < MP ? ztA + (size_t)(mp + 1) * SZ_FRAG : (has_b ? ztB : rnext), lane, nxt);
                    sz_colpass<FP16, NT>(Z[mp], UAh, UAl, w1h, w1l, cur);
                }
            }
            if (has_b) {
                uint32_t UBh[2 * SZ_RB], UBl[2 * SZ_RB];
#pragma unroll
                for (int rb = 0; rb < SZ_RB; ++rb) {
                    const uint4 v = ubw[rb * 64];
                    UBh[2 * rb] = v.x;
                    UBh[2 * rb + 1] = v.y;
                    UBl[2 * rb] = v.z;
                    UBl[2 * rb + 1] = v.w;
                }
                uint4 w1h[SZ_OB / 2], w1l[SZ_OB / 2];
                sz_phase1_windows(UBh, UBl, w1h, w1l);
#pragma unroll
                for (int mp = 0; mp < MP; ++mp) {
#pragma unroll
                    for (int c = 0; c < 2; ++c)
#pragma unroll
                        for (int hl = 0; hl < 2; ++hl) cur[c][hl] = nxt[c][hl];
                    sz_load_tab(mp + 1 < MP ? ztB + (size_t)(mp + 1) * SZ_FRAG : rnext, lane, nxt);
                    sz_colpass<FP16, NT>(Z[mp], UBh, UBl, w1h, w1l, cur);
                }
            }
#pragma unroll
            for (int c = 0; c < 2; ++c)
#pragma unroll
                for (int hl = 0; hl < 2; ++hl) cur[c][hl] = nxt[c][hl];
        }

        // ---- epilogue.  Lane (g4, j16) holds Z_m, m = 2 mp + g4 / 2, at rows
        // 8 ob + 4 (g4 mod 2) + e of column j16 of its strip.  Lanes g4 and
        // g4 ^ 2 hold the two halves of the same pixels: lane groups 0, 1 finish
        // the first half of the output blocks, groups 2, 3 the second.
        constexpr int HB = SZ_OB / 2;
        const bool lowg = g4 < 2;
        const int x = X0 + 16 * w + j16;
        // I at the pixels this lane finishes, requested before the vector work
        // below from clamped addresses (values past the image are loaded but
        // never used), so that its latency overlaps it; without I, R stands in
        // for the loads
        float iv[HB][4];
        {
            const float* ip = a.I ? a.I : a.X;
            const int xc = min(x, a.W - 1);
#pragma unroll
            for (int q = 0; q < HB; ++q)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int y = Y0 + 8 * (q + (lowg ? 0 : HB)) + 4 * (g4 & 1) + e;
                    iv[q][e] = ip[(size_t)min(y, a.H - 1) * a.W + xc];
                }
        }

        const double xh = a.sx * x + a.ox;
        const float xf = (float)xh;
        // per-lane weights of the spatial terms: P_m Z_m = (zinv_m xh^p) yh^q Z_m
        float wq[MP][3];
#pragma unroll
        for (int mp = 0; mp < MP; ++mp) {
            const int m = 2 * mp + (g4 >> 1);
            // (p, q) of term m: total degree tt, q = m - tt (tt + 1) / 2, p = tt - q
            const int tt = m >= 3 ? 2 : (m >= 1 ? 1 : 0);
            const int q = m - tt * (tt + 1) / 2, p = tt - q;
            const float c = ep[m] * (p == 0 ? 1.f : (p == 1 ? xf : xf * xf));
#pragma unroll
            for (int qq = 0; qq < 3; ++qq) wq[mp][qq] = (q == qq) ? c : 0.f;
        }
        float part[SZ_OB][4];
#pragma unroll
        for (int ob = 0; ob < SZ_OB; ++ob)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int y = Y0 + 8 * ob + 4 * (g4 & 1) + e;
                const float yf = fmaf((float)a.sy, (float)y, (float)a.oy);
                float v0 = 0.f, v1 = 0.f, v2 = 0.f;
#pragma unroll
                for (int mp = 0; mp < MP; ++mp) {
                    v0 = fmaf(wq[mp][0], Z[mp][ob][e], v0);
                    v1 = fmaf(wq[mp][1], Z[mp][ob][e], v1);
                    v2 = fmaf(wq[mp][2], Z[mp][ob][e], v2);
                }
                part[ob][e] = fmaf(fmaf(v2, yf, v1), yf, v0);
            }
        float fin[HB][4];
#pragma unroll
        for (int q = 0; q < HB; ++q)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const float send = lowg ? part[q + HB][e] : part[q][e];
                const float recv = __shfl_xor(send, 32);
                fin[q][e] = (lowg ? part[q][e] : part[q + HB][e]) + recv;
            }
        if (x < a.W) {
            // D = sum_m P_m Z_m - I + s sum_m gamma_m P_m (the pedestal restore),
            // in float32: sum_m P_m Z_m - I is exact where both are large (they
            // agree to a factor 2), and the rest is of the sky's size
            const float cy0 = fmaf(fmaf(ep[8 + 3], xf, ep[8 + 1]), xf, ep[8 + 0]);
            const float cy1 = fmaf(ep[8 + 4], xf, ep[8 + 2]);
            const float cy2 = ep[8 + 5];
            const bool has_i = a.I != nullptr;
#pragma unroll
            for (int q = 0; q < HB; ++q)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int ob = q + (lowg ? 0 : HB);
                    const int y = Y0 + 8 * ob + 4 * (g4 & 1) + e;
                    if (y < y_end) {
                        const float yf = fmaf((float)a.sy, (float)y, (float)a.oy);
                        const float pg = fmaf(fmaf(cy2, yf, cy1), yf, cy0);
                        a.out[(size_t)y * a.W + x] = fmaf(a.ped, pg, fin[q][e] - (has_i ? iv[q][e] : 0.f));
                    }
                }
        }

        // the next tile's samples (their registers would not fit beside Z);
        // once every wave is done with the staged tile, stage them.  Loads,
        // barrier and stores sit under one branch (`more` is uniform), so the
        // samples are not live across the passes.
        if (more) {
            float sv[SZ_SROWS][2];
            sz_load_tile(a, tn, ws, lane, sv);
            __syncthreads();
            sz_store_tile<FP16>(a, tn, ws, lane, sv, xs);
            __syncthreads();
        } else {
            __syncthreads();
        }
    }
}

template <bool FP16, int NT>
static int launch_sepz_p(const SepZArgs& a, int grid, hipStream_t s) {
    const int MP = (a.M + 1) / 2;
    if (MP <= 1)
        hipLaunchKernelGGL((contract_sepz_kernel<FP16, NT, 1>), dim3(grid), dim3(SZ_NT), SZ_LDS, s, a);
    else if (MP == 2)
        hipLaunchKernelGGL((contract_sepz_kernel<FP16, NT, 2>), dim3(grid), dim3(SZ_NT), SZ_LDS, s, a);
    else
        hipLaunchKernelGGL((contract_sepz_kernel<FP16, NT, 3>), dim3(grid), dim3(SZ_NT), SZ_LDS, s, a);
    return hip_status(hipGetLastError(), "contract_sepz_kernel");
}

// Compute units of the current device (cached per device).
static int device_cus() {
    static int cus[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (!cus[dev]) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
        cus[dev] = n;
    }
    return cus[dev];
}

int launch_contract_sepz(SepZArgs a, int precision, hipStream_t s) {
    if (a.h < 1 || a.h > kSepZMaxHalfWidth)
        return fail(SVCONV_EUNSUPPORTED, "regrouped separable form needs 1 <= half-width <= 12");
    if (a.M > 6) return fail(SVCONV_EUNSUPPORTED, "regrouped separable form needs spatial degree <= 2");
    a.tiles_x = (a.W + SZ_TW - 1) / SZ_TW;
    a.n_tiles = a.tiles_x * ((a.n_rows + SZ_TH - 1) / SZ_TH);
    if (a.n_tiles == 0) return SVCONV_OK;
    // persistent workgroups: SZ_MINW per compute unit (one 4-wave workgroup per
    // wave slot of a SIMD the registers allow), each walking its share of the tiles
    const int slots = SZ_MINW * device_cus();
    const int grid = a.n_tiles < slots ? a.n_tiles : slots;
    switch (precision) {
        case SVCONV_FP16X3: return launch_sepz_p<true, 3>(a, grid, s);
        case SVCONV_BF16X3: return launch_sepz_p<false, 3>(a, grid, s);
        case SVCONV_FP16X2: return launch_sepz_p<true, 2>(a, grid, s);
        default: return fail(SVCONV_EUNSUPPORTED, "regrouped separable form needs a split 16-bit precision");
    }
}

}  // namespace svc
