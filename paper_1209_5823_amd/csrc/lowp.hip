// Low-precision matrix-core contraction (bf16 / fp16 inputs, fp32
// accumulation) of the weighted multi-filter correlation
//
//   out(p) = sum_f w_f(p) T_f(p) - I(p),  T_f(p) = sum_{dv,du} F_f[dv][du] X(p + (du-h, dv-h)),
//
// with the optional hi + lo splits that recover precision:
//   X - ped = Xh + Xl,  F s_f = Fh + Fl  (each part rounded to nearest even),
//   T_f ~ (Fh.Xh + Fh.Xl + Fl.Xh) / s_f            (bf16x3, fp16x3)
//   T_f ~ (Fh.Xh + Fh.Xl) / s_f                    (fp16x2)
// s_f is a power of two per filter (fp16 only, to keep small taps normal)
// and X is scaled by 1/4 in fp16 so that 16-bit ADC counts stay finite.
//
// Matrix-core layout (v_mfma_f32_16x16x32_{bf16,f16}): the 32-long reduction
// of one instruction is 4 kernel rows (dv = 4r + g, lane group g) times 8
// consecutive kernel columns (du = 8q .. 8q+7).  B-operand lane (g, j) then
// needs 8 consecutive input samples of one LDS row: the 16 pixels of an
// instruction are 16 consecutive image rows at one column x, and every wave
// of the 8-wave workgroup owns the columns with one residue s = x mod 8, so
// its 8-sample windows start at the same misalignment s.  Each lane loads
// aligned 16-byte chunks of its row once per row group and funnel-shifts
// them into windows (v_alignbit), so the LDS reads are all aligned b128.
#include <cstdlib>

#include "internal.hpp"

namespace svc {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));

constexpr int LP_TP = 4;     // 16-pixel blocks per wave (columns x = X0 + s + 8 i)
constexpr int LP_NQ = 4;     // max 8-column chunks per kernel row (k <= 31)
constexpr int LP_WAVES = 8;  // one wave per column residue s
constexpr int LP_TW = 8 * LP_TP;
constexpr int LP_TH = 16;
constexpr float FP16_XSCALE = 0.25f;

__device__ __forceinline__ uint32_t f2bf_rne(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return u >> 16;
}
__device__ __forceinline__ float bf2f(uint32_t b) { return __uint_as_float(b << 16); }
__device__ __forceinline__ uint32_t f2h_rne(float x) {
    _Float16 v = (_Float16)x;
    return (uint32_t)__builtin_bit_cast(uint16_t, v);
}
__device__ __forceinline__ float h2f(uint32_t b) {
    return (float)__builtin_bit_cast(_Float16, (uint16_t)b);
}

template <bool FP16>
__device__ __forceinline__ void split16(float x, uint32_t& hi, uint32_t& lo) {
    if (FP16) {
        hi = f2h_rne(x);
        lo = f2h_rne(x - h2f(hi));
    } else {
        hi = f2bf_rne(x);
        lo = f2bf_rne(x - bf2f(hi));
    }
}

static int lp_pitch(int cols) {
    // 8-element (16-byte) units per row, odd so that the 16 rows read by one
    // b128 instruction fall in distinct bank groups
    int u = (cols + 7) / 8;
    if ((u & 1) == 0) ++u;
    return 8 * u;
}

LowpGeometry lowp_geometry(int k, int nb) {
    LowpGeometry g;
    g.k = k;
    g.n_rg = (k + 3) / 4;
    g.n_q = (k + 7) / 8;
    g.n_steps = g.n_rg * g.n_q;
    g.nb = nb;
    g.tile_w = LP_TW;
    g.tile_h = LP_TH;
    g.lds_rows = LP_TH + 4 * g.n_rg - 1;
    g.lds_pitch = lp_pitch(8 * (LP_TP + LP_NQ));
    const size_t tile = (size_t)g.lds_rows * g.lds_pitch * 2 * 2;                // hi + lo
    const size_t slab = (size_t)g.n_q * nb * 2 * 64 * 16;                        // one row group
    g.lds_bytes = tile + 2 * slab + (size_t)kMaxSpatialTerms * 4;
    return g;
}

size_t lowp_fragment_elems(int k, int nb) {
    const int n_rg = (k + 3) / 4, n_q = (k + 7) / 8;
    return (size_t)n_rg * n_q * nb * 2 * 64 * 8;   // hi and lo halves, 8 per lane
}

// Power-of-two scale per filter so that max |F_f| s_f lies in [1, 2) (fp16);
// inv[f] = 1 / (s_f xscale) restores the true T_f.  bf16 needs no scale.
__global__ void lowp_scale_kernel(const float* __restrict__ F, int NF, int kk, int fp16,
                                  float* __restrict__ scale, float* __restrict__ inv) {
    const int f = blockIdx.x;
    __shared__ float red[256];
    float m = 0.f;
    for (int q = threadIdx.x; q < kk; q += blockDim.x) m = fmaxf(m, fabsf(F[(size_t)f * kk + q]));
    red[threadIdx.x] = m;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        float sc = 1.f, xs = 1.f;
        if (fp16) {
            xs = FP16_XSCALE;
            const float mx = red[0];
            if (mx > 0.f) sc = ldexpf(1.f, -ilogbf(mx));
        }
        scale[f] = sc;
        if (inv) inv[f] = 1.f / (sc * xs);
    }
}

// A-operand fragments: element e of lane l, block b, row group r, chunk q is
// filter f = 16 b + (l & 15) at (dv = 4 r + (l >> 4), du = 8 q + e), scaled.
// Packed (at most 8 filters, one block): rows 0..7 are filters 0..7 at du,
// rows 8..15 the same filters at du - 1, i.e. the taps of the next output
// column on the same input window.  Layout [r][q][b][half][lane][8], half 0 =
// hi, 1 = lo.
__global__ void frag_lowp_kernel(const float* __restrict__ F, const float* __restrict__ scale,
                                 int NF, int k, int nb, int n_rg, int n_q, int fp16, int packed,
                                 uint16_t* __restrict__ frag) {
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;   // one (r,q,b,lane,e)
    const long total = (long)n_rg * n_q * nb * 64 * 8;
    if (idx >= total) return;
    const int e = (int)(idx & 7);
    const int lane = (int)((idx >> 3) & 63);
    long rest = idx >> 9;
    const int b = (int)(rest % nb);
    rest /= nb;
    const int q = (int)(rest % n_q);
    const int r = (int)(rest / n_q);
    const int fl = lane & 15;
    const int f = packed ? (fl & 7) : 16 * b + fl;
    const int dv = 4 * r + (lane >> 4);
    const int du = 8 * q + e - (packed ? (fl >> 3) : 0);
    float v = 0.f;
    if (f < NF && dv < k && du >= 0 && du < k) v = F[((size_t)f * k + dv) * k + du] * scale[f];
    uint32_t hi, lo;
    if (fp16) split16<true>(v, hi, lo);
    else split16<false>(v, hi, lo);
    const size_t base = ((((size_t)(r * n_q + q) * nb + b) * 2) * 64 + lane) * 8 + e;
    frag[base] = (uint16_t)hi;
    frag[base + 64 * 8] = (uint16_t)lo;
}

int build_lowp_fragments(const float* F, int NF, int k, int fp16, float* scale,
                         uint16_t* frag, hipStream_t s, bool packed) {
    // scale: 2 * kMaxFilters floats, [0, kMaxFilters) the scales s_f and
    // [kMaxFilters, 2 kMaxFilters) the inverse factors used by the epilogue
    if (k > 8 * LP_NQ) return SVCONV_OK;   // beyond the low-precision kernel's reach
    const int nb = (NF + 15) / 16;
    const int n_rg = (k + 3) / 4, n_q = (k + 7) / 8;
    hipLaunchKernelGGL(lowp_scale_kernel, dim3(NF), dim3(256), 0, s, F, NF, k * k, fp16, scale,
                       scale + kMaxFilters);
    int st = hip_status(hipGetLastError(), "lowp_scale_kernel");
    if (st) return st;
    const long total = (long)n_rg * n_q * nb * 64 * 8;
    hipLaunchKernelGGL(frag_lowp_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, F,
                       scale, NF, k, nb, n_rg, n_q, fp16, packed ? 1 : 0, frag);
    return hip_status(hipGetLastError(), "frag_lowp_kernel");
}

// ------------------------------------------------------------ contraction --

// W_t = samples [s, s+8) of chunk_t ++ chunk_{t+1}; S2 = s / 2, sh = 16 (s & 1).
template <int S2, int NW>
__device__ __forceinline__ void form_windows(uint32_t (&c)[NW + 1][4], uint32_t sh) {
#pragma unroll
    for (int t = 0; t < NW; ++t) {
        uint32_t d[8];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            d[e] = c[t][e];
            d[e + 4] = c[t + 1][e];
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) c[t][e] = __builtin_amdgcn_alignbit(d[e + S2 + 1], d[e + S2], sh);
    }
}

template <bool FP16>
__device__ __forceinline__ f4 mfma16(const uint32_t (&a)[4], const uint32_t (&b)[4], f4 c) {
    if constexpr (FP16) {
        h8 av = __builtin_bit_cast(h8, a);
        h8 bv = __builtin_bit_cast(h8, b);
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(av, bv, c, 0, 0, 0);
    } else {
        bf8 av = __builtin_bit_cast(bf8, a);
        bf8 bv = __builtin_bit_cast(bf8, b);
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, c, 0, 0, 0);
    }
}

// Stage rows [r0, r1) of the input tile, (X - ped) * xscale split into
// 16-bit hi / lo parts, X = 0 outside the image.  Tile row r is image row
// Y0 - h + r, tile column c is image column X0 - h + c.
template <bool FP16, bool SPLIT_R>
__device__ __forceinline__ void lp_stage(const ContractArgs& a, uint16_t* hiT, uint16_t* loT,
                                         int pitch, int rows, int X0, int Y0, float xscale,
                                         int tid) {
    // element pairs, one 32-bit LDS word per part (pitch is even)
    const int cols = 8 * (LP_TP + LP_NQ);
    const int half = pitch / 2;
    for (int r = tid >> 6; r < rows; r += LP_WAVES) {
        const int gy = Y0 - a.h + r;
        const bool row_in = (gy >= 0) && (gy < a.H);
        const float* src = a.X + (size_t)(row_in ? gy : 0) * a.W;
        for (int c2 = tid & 63; c2 < half; c2 += 64) {
            // both loads from clamped addresses, the masks applied after
            float xr[2];
#pragma unroll
            for (int v = 0; v < 2; ++v) {
                const int gx = X0 - a.h + 2 * c2 + v;
                xr[v] = src[gx < 0 ? 0 : (gx < a.W ? gx : a.W - 1)];
            }
            uint32_t hw = 0, lw = 0;
#pragma unroll
            for (int v = 0; v < 2; ++v) {
                const int c = 2 * c2 + v;
                const int gx = X0 - a.h + c;
                const float x = (row_in && gx >= 0 && gx < a.W) ? xr[v] : 0.f;
                const float xv = (c < cols) ? (x - a.ped) * xscale : 0.f;
                uint32_t hi, lo;
                split16<FP16>(xv, hi, lo);
                hw |= hi << (16 * v);
                lw |= (SPLIT_R ? lo : 0u) << (16 * v);
            }
            reinterpret_cast<uint32_t*>(hiT + r * pitch)[c2] = hw;
            reinterpret_cast<uint32_t*>(loT + r * pitch)[c2] = lw;
        }
    }
}

// One 4-row group r of the contraction for this wave's 4 pixel blocks:
// windows from LDS row (j + 4r + g), A fragments of chunk q from `sl`
// ([q][b][half][lane] 16-byte units), the next chunk's fragments loaded while
// this chunk's products run.  `hook(q)` runs once per chunk (used to stream
// the next slab in the slab kernel).
template <int NB, bool FP16, bool SPLIT_R, bool SPLIT_B, class Hook>
__device__ __forceinline__ void lp_rowgroup(f4 (&acc)[NB][LP_TP], const uint16_t* hiT,
                                            const uint16_t* loT, int pitch, int row,
                                            const uint4* sl, int n_q, int lane, int s,
                                            Hook&& hook) {
    constexpr int HALVES = SPLIT_B ? 2 : 1;
    constexpr int NCH = LP_TP + LP_NQ;
    const uint32_t sh = 16u * (uint32_t)(s & 1);
    uint32_t ch[NCH][4], cl[NCH][4];
    {
        const uint4* ph = reinterpret_cast<const uint4*>(hiT + row * pitch);
        const uint4* pl = reinterpret_cast<const uint4*>(loT + row * pitch);
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const uint4 vh = ph[c];
            ch[c][0] = vh.x; ch[c][1] = vh.y; ch[c][2] = vh.z; ch[c][3] = vh.w;
            if (SPLIT_R) {
                const uint4 vl = pl[c];
                cl[c][0] = vl.x; cl[c][1] = vl.y; cl[c][2] = vl.z; cl[c][3] = vl.w;
            }
        }
    }
    switch (s >> 1) {
        case 0: form_windows<0, NCH - 1>(ch, sh); if (SPLIT_R) form_windows<0, NCH - 1>(cl, sh); break;
        case 1: form_windows<1, NCH - 1>(ch, sh); if (SPLIT_R) form_windows<1, NCH - 1>(cl, sh); break;
        case 2: form_windows<2, NCH - 1>(ch, sh); if (SPLIT_R) form_windows<2, NCH - 1>(cl, sh); break;
        default: form_windows<3, NCH - 1>(ch, sh); if (SPLIT_R) form_windows<3, NCH - 1>(cl, sh); break;
    }

    uint32_t fh[NB][4], fl[NB][4];
    auto load_frags = [&](int q, uint32_t (&h_)[NB][4], uint32_t (&l_)[NB][4]) {
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const uint4 vh = sl[((q * NB + b) * HALVES + 0) * 64 + lane];
            h_[b][0] = vh.x; h_[b][1] = vh.y; h_[b][2] = vh.z; h_[b][3] = vh.w;
            if (SPLIT_B) {
                const uint4 vl = sl[((q * NB + b) * HALVES + 1) * 64 + lane];
                l_[b][0] = vl.x; l_[b][1] = vl.y; l_[b][2] = vl.z; l_[b][3] = vl.w;
            }
        }
    };
    load_frags(0, fh, fl);
#pragma unroll
    for (int q = 0; q < LP_NQ; ++q) {
        if (q < n_q) {
            hook(q, 0);
            uint32_t nh[NB][4], nl[NB][4];
            if (q + 1 < n_q) load_frags(q + 1, nh, nl);
            // pass-outer order: NB * LP_TP independent accumulators between two
            // products that update the same one
#pragma unroll
            for (int b = 0; b < NB; ++b)
#pragma unroll
                for (int i = 0; i < LP_TP; ++i) acc[b][i] = mfma16<FP16>(fh[b], ch[i + q], acc[b][i]);
            if (SPLIT_R) {
#pragma unroll
                for (int b = 0; b < NB; ++b)
#pragma unroll
                    for (int i = 0; i < LP_TP; ++i) acc[b][i] = mfma16<FP16>(fh[b], cl[i + q], acc[b][i]);
            }
            if (SPLIT_B) {
#pragma unroll
                for (int b = 0; b < NB; ++b)
#pragma unroll
                    for (int i = 0; i < LP_TP; ++i) acc[b][i] = mfma16<FP16>(fl[b], ch[i + q], acc[b][i]);
            }
            if (q + 1 < n_q) {
#pragma unroll
                for (int b = 0; b < NB; ++b)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        fh[b][e] = nh[b][e];
                        if (SPLIT_B) fl[b][e] = nl[b][e];
                    }
            }
            hook(q, 1);
        }
    }
}

// I at the lane's pixels, all requested together from clamped addresses (X
// stands in when there is no I); values of pixels outside the band, or with
// no I, are never used.
template <int N>
__device__ __forceinline__ void lp_fetch_i(const ContractArgs& a, float (&iv)[N], int x0, int dx,
                                           int y) {
    const float* ip = a.I ? a.I : a.X;
    const int y_last = a.y_begin + a.n_rows - 1;
    const size_t row = (size_t)(y < y_last ? y : y_last) * a.W;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const int x = x0 + dx * i;
        iv[i] = ip[row + (x < a.W ? x : a.W - 1)];
    }
}

// x^e for 0 <= e <= 7 from the binary digits of e (no branches)
__device__ __forceinline__ float lp_pow(float x, float x2, float x4, int e) {
    return ((e & 1) ? x : 1.f) * ((e & 2) ? x2 : 1.f) * ((e & 4) ? x4 : 1.f);
}

// Epilogue.  With U_m(p) = sum_f coef[f][m] T_f(p) / (s_f xscale) and
// gamma_m = sum_f coef[f][m] beta_f,
//   out(p) = sum_m P_m(p) (U_m(p) + ped gamma_m) - I(p)
// (regrouped form: coef = identity).  U for one 16-pixel block is a
// (16 terms x 64 filters) . (64 filters x 16 pixels) product on the float32
// matrix cores: accumulator register (b, e) of lane (g, j) is T_f for
// f = 16 b + 4 g + e at pixel j, which is exactly the B operand of
// v_mfma_f32_16x16x4_f32 with K index g, so no data moves between lanes.
// A operand (b, e, mb): lane (k, m_l) holds coef[16 b + 4 k + e][16 mb + m_l] / (s_f xscale).
// The result U[m][j] sits in lane (g, j), register e' for m = 16 mb + 4 g + e'.
// float32 throughout: its rounding (~1e-7 relative) is far below the
// tolerance of the 16-bit forms.
template <int NB, int MB>
__device__ __forceinline__ void lp_epilogue(const ContractArgs& a, const f4 (&acc)[NB][LP_TP],
                                            const float (&afr)[NB][4][MB],
                                            const float* gamma_s, int X0, int Y0, int s, int g,
                                            int j) {
    // I at the lane's pixels, requested first so that the matrix-core work
    // below hides its latency (the contraction's registers are free by now)
    float iv[LP_TP];
    const int y = Y0 + j;
    lp_fetch_i(a, iv, X0 + s, 8, y);
    const float yh = (float)(a.sy * y + a.oy);
    // exponents of the lane's four terms per term block
    // and the y power of each, formed once
    int ei[MB][4];
    float py[MB][4];
    {
        const float yh2 = yh * yh, yh4 = yh2 * yh2;
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int m = 16 * mb + 4 * g + e;
                int tt = 0;
                while ((tt + 1) * (tt + 2) / 2 <= m) ++tt;
                const int ej = m - tt * (tt + 1) / 2;
                ei[mb][e] = tt - ej;
                py[mb][e] = lp_pow(yh, yh2, yh4, ej);
            }
    }
#pragma unroll
    for (int i = 0; i < LP_TP; ++i) {
        f4 u[MB];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) u[mb] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if (16 * b + e < a.NF)   // else filters 16 b + 4 k + e are all padding
#pragma unroll
                    for (int mb = 0; mb < MB; ++mb)
                        u[mb] = __builtin_amdgcn_mfma_f32_16x16x4f32(afr[b][e][mb], acc[b][i][e], u[mb], 0, 0, 0);
        const int x = X0 + s + 8 * i;
        const float xh = (float)(a.sx * x + a.ox), xh2 = xh * xh, xh4 = xh2 * xh2;
        float part = 0.f;
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int m = 16 * mb + 4 * g + e;
                if (m < a.M)
                    part += lp_pow(xh, xh2, xh4, ei[mb][e]) * py[mb][e] * (u[mb][e] + a.ped * gamma_s[m]);
            }
        part += __shfl_xor(part, 16);
        part += __shfl_xor(part, 32);
        if (g == 0 && x < a.W && y < a.y_begin + a.n_rows)
            a.out[(size_t)y * a.W + x] = part - (a.I ? iv[i] : 0.f);
    }
}

// Prologue of the epilogue: A fragments of the U product and gamma (in LDS).
template <int NB, int MB, bool REG>
__device__ __forceinline__ void lp_epilogue_setup(const ContractArgs& a, float (&afr)[NB][4][MB],
                                                  float* gamma_s, int tid, int lane) {
    const int k = lane >> 4, ml = lane & 15;
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) {
                // loads from clamped indices, masked after (no load under a branch)
                const int f = 16 * b + 4 * k + e;
                const int m = 16 * mb + ml;
                const int fc = f < a.NF ? f : a.NF - 1, mc = m < a.M ? m : a.M - 1;
                const float inv = a.fscale ? a.fscale[fc] : 1.f;
                const float c = REG ? (f == m ? 1.f : 0.f) : a.coef[fc * a.M + mc];
                afr[b][e][mb] = (f < a.NF && m < a.M) ? c * inv : 0.f;
            }
    if (tid < a.M) {
        double gm = 0.0;
        if (a.beta) {
            if (REG) {
                gm = a.beta[tid];
            } else {
                for (int f = 0; f < a.NF; ++f) gm += (double)a.coef[f * a.M + tid] * a.beta[f];
            }
        }
        gamma_s[tid] = (float)gm;
    }
}

// ------------------------------------------- two-column packed contraction --
//
// With at most 8 filters (the regrouped form's M <= 8) half of a 16-row A
// operand would be empty.  Packed, rows 8..15 hold the same filters shifted by
// one kernel column, so each product yields the filters at two neighbouring
// output columns x and x + 1 from one input window: wave w owns the column
// pairs (2 w + 16 i, 2 w + 16 i + 1), i < LP_TP / 2, and issues half the
// products.  The windows then start at an even sample, 2 w mod 8, i.e. on a
// 32-bit word: no funnel shifts.
constexpr int LP_PB = LP_TP / 2;                 // column pairs per wave
constexpr int LP_PNCH = 2 * LP_PB + LP_NQ - 1;   // 16-byte chunks a packed lane loads per row

// windows W_t = words [D, D + 4) of chunk t ++ chunk t + 1, formed in place
template <int D>
__device__ __forceinline__ void lp_word_windows(uint32_t (&c)[LP_PNCH][4]) {
#pragma unroll
    for (int t = 0; t + 1 < LP_PNCH; ++t)
#pragma unroll
        for (int e = 0; e < 4; ++e) c[t][e] = (e + D < 4) ? c[t][e + D] : c[t + 1][e + D - 4];
}

template <bool FP16, bool SPLIT_R, bool SPLIT_B>
__device__ __forceinline__ void lp_rowgroup_packed(f4 (&acc)[LP_PB], const uint16_t* hiT,
                                                   const uint16_t* loT, int pitch, int row,
                                                   const uint4* sl, int n_q, int lane, int w) {
    constexpr int HALVES = SPLIT_B ? 2 : 1;
    const int cb = w >> 2;   // the chunk that holds sample 2 w
    uint32_t ch[LP_PNCH][4], cl[LP_PNCH][4];
    {
        const uint4* ph = reinterpret_cast<const uint4*>(hiT + row * pitch) + cb;
        const uint4* pl = reinterpret_cast<const uint4*>(loT + row * pitch) + cb;
#pragma unroll
        for (int c = 0; c < LP_PNCH; ++c) {
            const uint4 vh = ph[c];
            ch[c][0] = vh.x; ch[c][1] = vh.y; ch[c][2] = vh.z; ch[c][3] = vh.w;
            if (SPLIT_R) {
                const uint4 vl = pl[c];
                cl[c][0] = vl.x; cl[c][1] = vl.y; cl[c][2] = vl.z; cl[c][3] = vl.w;
            }
        }
    }
    switch (w & 3) {
        case 0: break;
        case 1: lp_word_windows<1>(ch); if (SPLIT_R) lp_word_windows<1>(cl); break;
        case 2: lp_word_windows<2>(ch); if (SPLIT_R) lp_word_windows<2>(cl); break;
        default: lp_word_windows<3>(ch); if (SPLIT_R) lp_word_windows<3>(cl); break;
    }
    uint32_t fh[4], fl[4];
    auto load_frags = [&](int q, uint32_t (&h_)[4], uint32_t (&l_)[4]) {
        const uint4 vh = sl[(q * HALVES + 0) * 64 + lane];
        h_[0] = vh.x; h_[1] = vh.y; h_[2] = vh.z; h_[3] = vh.w;
        if (SPLIT_B) {
            const uint4 vl = sl[(q * HALVES + 1) * 64 + lane];
            l_[0] = vl.x; l_[1] = vl.y; l_[2] = vl.z; l_[3] = vl.w;
        }
    };
    load_frags(0, fh, fl);
#pragma unroll
    for (int q = 0; q < LP_NQ; ++q) {
        if (q < n_q) {
            uint32_t nh[4], nl[4];
            if (q + 1 < n_q) load_frags(q + 1, nh, nl);
#pragma unroll
            for (int i = 0; i < LP_PB; ++i) acc[i] = mfma16<FP16>(fh, ch[2 * i + q], acc[i]);
            if (SPLIT_R)
#pragma unroll
                for (int i = 0; i < LP_PB; ++i) acc[i] = mfma16<FP16>(fh, cl[2 * i + q], acc[i]);
            if (SPLIT_B)
#pragma unroll
                for (int i = 0; i < LP_PB; ++i) acc[i] = mfma16<FP16>(fl, ch[2 * i + q], acc[i]);
            if (q + 1 < n_q)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    fh[e] = nh[e];
                    if (SPLIT_B) fl[e] = nl[e];
                }
        }
    }
}

// A fragments of the packed epilogue's U product: lane (k, m_l) holds, for
// register e of the contraction, 1 / (s_f xscale) when filter f = 4 (k & 1) +
// e is term m = m_l & 7 of the same output column (m_l >> 3 == k >> 1).
__device__ __forceinline__ void lp_epilogue_setup_packed(const ContractArgs& a, float (&afr)[4], int lane) {
    const int k = lane >> 4, ml = lane & 15;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int f = 4 * (k & 1) + e, m = ml & 7;
        float v = 0.f;
        if ((ml >> 3) == (k >> 1) && f == m && f < a.NF && m < a.M) v = a.fscale ? a.fscale[f] : 1.f;
        afr[e] = v;
    }
}

// Packed epilogue (regrouped form): lane (g, j) register e holds T_f, f =
// 4 (g & 1) + e, at column x_i + (g >> 1), x_i = X0 + 2 w + 16 i, row Y0 + j;
// the U product leaves U_m of column x_i in lane groups 0, 1 and of x_i + 1 in
// groups 2, 3 (m = 4 (g & 1) + e').
__device__ __forceinline__ void lp_epilogue_packed(const ContractArgs& a, const f4 (&acc)[LP_PB],
                                                   const float (&afr)[4], const float* gamma_s, int X0,
                                                   int Y0, int w, int g, int j) {
    const int y = Y0 + j;
    const int xoff = 2 * w + (g >> 1);
    float iv[LP_PB];
    lp_fetch_i(a, iv, X0 + xoff, 16, y);
    const float yh = (float)(a.sy * y + a.oy), yh2 = yh * yh, yh4 = yh2 * yh2;
    // x exponent and y power of the lane's four terms
    int ei[4];
    float py[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int m = 4 * (g & 1) + e;
        int tt = 0;
        while ((tt + 1) * (tt + 2) / 2 <= m) ++tt;
        const int ej = m - tt * (tt + 1) / 2;
        ei[e] = tt - ej;
        py[e] = lp_pow(yh, yh2, yh4, ej);
    }
#pragma unroll
    for (int i = 0; i < LP_PB; ++i) {
        f4 u = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int e = 0; e < 4; ++e) u = __builtin_amdgcn_mfma_f32_16x16x4f32(afr[e], acc[i][e], u, 0, 0, 0);
        const int x = X0 + xoff + 16 * i;
        const float xh = (float)(a.sx * x + a.ox), xh2 = xh * xh, xh4 = xh2 * xh2;
        float part = 0.f;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int m = 4 * (g & 1) + e;
            if (m < a.M) part += lp_pow(xh, xh2, xh4, ei[e]) * py[e] * (u[e] + a.ped * gamma_s[m]);
        }
        part += __shfl_xor(part, 16);
        if ((g & 1) == 0 && x < a.W && y < a.y_begin + a.n_rows)
            a.out[(size_t)y * a.W + x] = part - (a.I ? iv[i] : 0.f);
    }
}

__device__ __forceinline__ int lp_xcd_remap(int bid, int n) {
    const int x8 = bid & 7, tt = bid >> 3, q8 = n >> 3, r8 = n & 7;
    return x8 * q8 + (x8 < r8 ? x8 : r8) + tt;
}

// Slab kernel: one tile per workgroup; the A fragments of one 4-row group at a
// time sit in a double-buffered LDS slab, the next group's slab streamed in
// one chunk per q iteration.  Used when the whole fragment table does not
// fit in LDS (large kernels).
template <int NB, int MB, bool FP16, bool SPLIT_R, bool SPLIT_B, bool REG>
__global__ __launch_bounds__(512, 1) void contract_lowp_kernel(
    ContractArgs a, const uint16_t* __restrict__ frag, int k, int n_rg, int n_q, int pitch,
    int rows, int tiles_x, int n_tiles, float xscale) {
    extern __shared__ __align__(16) uint8_t smem_raw[];
    constexpr int HALVES = SPLIT_B ? 2 : 1;
    uint16_t* hiT = reinterpret_cast<uint16_t*>(smem_raw);
    uint16_t* loT = hiT + rows * pitch;
    uint4* slab = reinterpret_cast<uint4*>(loT + rows * pitch);
    const int slab_u4 = n_q * NB * HALVES * 64;
    float* gamma_s = reinterpret_cast<float*>(slab + 2 * slab_u4);

    const int tid = threadIdx.x;
    const int t = lp_xcd_remap(blockIdx.x, n_tiles);
    const int X0 = (t % tiles_x) * LP_TW;
    const int Y0 = a.y_begin + (t / tiles_x) * LP_TH;

    float afr[NB][4][MB];
    lp_epilogue_setup<NB, MB, REG>(a, afr, gamma_s, tid, tid & 63);
    lp_stage<FP16, SPLIT_R>(a, hiT, loT, pitch, rows, X0, Y0, xscale, tid);

    // slab of row group r: [q][b][half][lane] 16-byte units
    auto slab_src = [&](int r, int u) -> const uint4* {
        const int lane = u & 63;
        int rest = u >> 6;
        const int hf = rest % HALVES;
        rest /= HALVES;
        const int b = rest % NB;
        const int q = rest / NB;
        const size_t unit = (((size_t)(r * n_q + q) * NB + b) * 2 + hf) * 64 + lane;
        return reinterpret_cast<const uint4*>(frag) + unit;
    };
    for (int u = tid; u < slab_u4; u += 512) slab[u] = *slab_src(0, u);
    __syncthreads();

    const int lane = tid & 63, w = tid >> 6;
    const int g = lane >> 4, j = lane & 15;

    f4 acc[NB][LP_TP];
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int i = 0; i < LP_TP; ++i) acc[b][i] = f4{0.f, 0.f, 0.f, 0.f};

    constexpr int UPQ = NB * HALVES * 64;       // slab units of one chunk q (<= 512)
    for (int r = 0; r < n_rg; ++r) {
        // the next row group's slab is copied one chunk q per iteration (one
        // 16-byte unit per thread at most) into the buffer no wave reads now
        const bool more = (r + 1 < n_rg);
        uint4* dst = slab + ((r + 1) & 1) * slab_u4;
        const bool do_pf = more && tid < UPQ;
        uint4 pfq;
        auto hook = [&](int q, int phase) {
            if (!do_pf) return;
            if (phase == 0) pfq = *slab_src(r + 1, q * UPQ + tid);
            else dst[q * UPQ + tid] = pfq;
        };
        lp_rowgroup<NB, FP16, SPLIT_R, SPLIT_B>(acc, hiT, loT, pitch, j + 4 * r + g,
                                               slab + (r & 1) * slab_u4, n_q, lane, w, hook);
        __syncthreads();   // the next slab is complete and this one is free
    }
    lp_epilogue<NB, MB>(a, acc, afr, gamma_s, X0, Y0, w, g, j);
}

// Resident kernel: the whole A-fragment table lives in LDS and a persistent
// workgroup walks a contiguous run of tiles (one XCD's workgroups cover
// neighbouring runs); the next tile's input is loaded into registers while
// the current tile is contracted, so the only barriers are the two around
// each tile's staging.
constexpr int LP_PF = 4;   // staged element pairs per thread and tile (rows * pitch <= 1024 * LP_PF)

template <int NB, int MB, bool FP16, bool SPLIT_R, bool SPLIT_B, bool REG, bool PACK>
__global__ __launch_bounds__(512, 1) void contract_lowp_resident_kernel(
    ContractArgs a, const uint16_t* __restrict__ frag, int k, int n_rg, int n_q, int pitch,
    int rows, int tiles_x, int n_tiles, int tiles_per_wg, float xscale) {
    extern __shared__ __align__(16) uint8_t smem_raw[];
    constexpr int HALVES = SPLIT_B ? 2 : 1;
    uint16_t* hiT = reinterpret_cast<uint16_t*>(smem_raw);
    uint16_t* loT = hiT + rows * pitch;
    uint4* table = reinterpret_cast<uint4*>(loT + rows * pitch);
    const int rg_u4 = n_q * NB * HALVES * 64;   // units of one row group
    float* gamma_s = reinterpret_cast<float*>(table + n_rg * rg_u4);

    const int tid = threadIdx.x;
    const int lane = tid & 63, w = tid >> 6;
    const int g = lane >> 4, j = lane & 15;
    const int wg = lp_xcd_remap(blockIdx.x, gridDim.x);
    const int t_begin = wg * tiles_per_wg;
    const int t_end = min(n_tiles, t_begin + tiles_per_wg);
    if (t_begin >= t_end) return;   // uniform for the workgroup

    float afr[NB][4][MB];
    lp_epilogue_setup<NB, MB, REG>(a, afr, gamma_s, tid, lane);
    float afp[4];
    if constexpr (PACK) lp_epilogue_setup_packed(a, afp, lane);
    // whole table: unit (r, q, b, hf, lane) from the [r][q][b][2][lane] global layout
    for (int u = tid; u < n_rg * rg_u4; u += 512) {
        const int ln = u & 63;
        int rest = u >> 6;
        const int hf = rest % HALVES;
        rest /= HALVES;
        const int b = rest % NB;
        rest /= NB;
        const int q = rest % n_q;
        const int r = rest / n_q;
        const size_t unit = (((size_t)(r * n_q + q) * NB + b) * 2 + hf) * 64 + ln;
        table[u] = reinterpret_cast<const uint4*>(frag)[unit];
    }

    // raw input of a tile: element pair (2 e, 2 e + 1), e = tid + 512 p, of
    // the rows x pitch tile (pitch is even), stored as one 32-bit word per part.
    // The loads go out together from clamped addresses; the masks (X = 0
    // outside the image) apply when the tile is stored.
    float pf[LP_PF][2];
    auto fetch = [&](int t) {
        const int X0 = (t % tiles_x) * LP_TW;
        const int Y0 = a.y_begin + (t / tiles_x) * LP_TH;
#pragma unroll
        for (int p = 0; p < LP_PF; ++p) {
            const int e2 = 2 * (tid + 512 * p);
            const int r = e2 / pitch, c = e2 - r * pitch;
            const int gy = Y0 - a.h + r, gx = X0 - a.h + c;
            const size_t row = (size_t)(gy < 0 ? 0 : (gy < a.H ? gy : a.H - 1)) * a.W;
#pragma unroll
            for (int v = 0; v < 2; ++v) {
                const int xv = gx + v;
                pf[p][v] = a.X[row + (xv < 0 ? 0 : (xv < a.W ? xv : a.W - 1))];
            }
        }
    };
    auto store = [&](int t) {
        const int X0 = (t % tiles_x) * LP_TW;
        const int Y0 = a.y_begin + (t / tiles_x) * LP_TH;
        const int cols = 8 * (LP_TP + LP_NQ);
#pragma unroll
        for (int p = 0; p < LP_PF; ++p) {
            const int e2 = 2 * (tid + 512 * p);
            const int r = e2 / pitch, c = e2 - r * pitch;
            if (r < rows) {
                const int gy = Y0 - a.h + r, gx = X0 - a.h + c;
                const bool row_in = gy >= 0 && gy < a.H;
                uint32_t hw = 0, lw = 0;
#pragma unroll
                for (int v = 0; v < 2; ++v) {
                    const bool in = row_in && gx + v >= 0 && gx + v < a.W;
                    const float xv = (c + v < cols) ? ((in ? pf[p][v] : 0.f) - a.ped) * xscale : 0.f;
                    uint32_t hi, lo;
                    split16<FP16>(xv, hi, lo);
                    hw |= hi << (16 * v);
                    lw |= (SPLIT_R ? lo : 0u) << (16 * v);
                }
                reinterpret_cast<uint32_t*>(hiT)[e2 >> 1] = hw;
                reinterpret_cast<uint32_t*>(loT)[e2 >> 1] = lw;
            }
        }
    };
    fetch(t_begin);
    for (int t = t_begin; t < t_end; ++t) {
        __syncthreads();           // previous tile's LDS reads are done
        store(t);
        __syncthreads();           // tile (and, first time, table) visible
        const int X0 = (t % tiles_x) * LP_TW;
        const int Y0 = a.y_begin + (t / tiles_x) * LP_TH;
        if (t + 1 < t_end) fetch(t + 1);
        if constexpr (PACK) {
            f4 acc[LP_PB];
#pragma unroll
            for (int i = 0; i < LP_PB; ++i) acc[i] = f4{0.f, 0.f, 0.f, 0.f};
            for (int r = 0; r < n_rg; ++r)
                lp_rowgroup_packed<FP16, SPLIT_R, SPLIT_B>(acc, hiT, loT, pitch, j + 4 * r + g,
                                                           table + r * rg_u4, n_q, lane, w);
            lp_epilogue_packed(a, acc, afp, gamma_s, X0, Y0, w, g, j);
        } else {
            f4 acc[NB][LP_TP];
#pragma unroll
            for (int b = 0; b < NB; ++b)
#pragma unroll
                for (int i = 0; i < LP_TP; ++i) acc[b][i] = f4{0.f, 0.f, 0.f, 0.f};
            auto nohook = [](int, int) {};
            for (int r = 0; r < n_rg; ++r)
                lp_rowgroup<NB, FP16, SPLIT_R, SPLIT_B>(acc, hiT, loT, pitch, j + 4 * r + g,
                                                       table + r * rg_u4, n_q, lane, w, nohook);
            lp_epilogue<NB, MB>(a, acc, afr, gamma_s, X0, Y0, w, g, j);
        }
    }
}

static int g_num_cus = 0;

static int num_cus() {
    if (g_num_cus == 0) {
        int dev = 0, n = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0)
            g_num_cus = n;
        else
            g_num_cus = 256;
    }
    return g_num_cus;
}

// Whether the persistent kernel with the whole fragment table in LDS runs for
// these arguments (else the slab kernel).
static bool lowp_resident(const ContractArgs& a, int nb, bool split_b, int* n_tiles_out = nullptr,
                          int* tiles_x_out = nullptr) {
    const int HALVES = split_b ? 2 : 1;
    const int k = 2 * a.h + 1;
    const LowpGeometry g = lowp_geometry(k, nb);
    const int tiles_x = (a.W + g.tile_w - 1) / g.tile_w;
    const int tiles_y = (a.n_rows + g.tile_h - 1) / g.tile_h;
    const int n_tiles = tiles_x * tiles_y;
    if (n_tiles_out) *n_tiles_out = n_tiles;
    if (tiles_x_out) *tiles_x_out = tiles_x;
    const size_t tile_bytes = (size_t)g.lds_rows * g.lds_pitch * 2 * 2;
    const size_t table_bytes = (size_t)g.n_rg * g.n_q * nb * HALVES * 64 * 16;
    const size_t coef_bytes = (size_t)kMaxSpatialTerms * 4;   // gamma
    const bool fits_pf = (size_t)g.lds_rows * g.lds_pitch <= (size_t)1024 * LP_PF;
    return tile_bytes + table_bytes + coef_bytes <= (size_t)160 * 1024 && fits_pf && n_tiles >= 2 * num_cus();
}

bool lowp_packed(const ContractArgs& a, int nb) {
    const int k = 2 * a.h + 1;
    // every split precision keeps the lo half of the fragments (SPLIT_B) except
    // fp16x2, whose table is half as large: the resident test with the larger
    // table holds for both
    return a.coef == nullptr && nb == 1 && a.M <= 8 && k <= 8 * LP_NQ && lowp_resident(a, nb, true);
}

template <int NB, int MB, bool FP16, bool SR, bool SB>
static int launch_lowp_t(const ContractArgs& a, const uint16_t* frag, bool reg, hipStream_t s) {
    const int k = 2 * a.h + 1;
    const LowpGeometry g = lowp_geometry(k, NB);
    int n_tiles = 0, tiles_x = 0;
    const bool resident = lowp_resident(a, NB, SB, &n_tiles, &tiles_x);
    if (n_tiles == 0) return SVCONV_OK;
    const float xs = FP16 ? FP16_XSCALE : 1.f;
    constexpr int HALVES = SB ? 2 : 1;
    const size_t resident_bytes = (size_t)g.lds_rows * g.lds_pitch * 2 * 2 +
                                  (size_t)g.n_rg * g.n_q * NB * HALVES * 64 * 16 + (size_t)kMaxSpatialTerms * 4;
    if (resident) {
        const int n_wg = num_cus();
        const int per = (n_tiles + n_wg - 1) / n_wg;
        if constexpr (NB == 1 && MB == 1) {
            if (lowp_packed(a, NB)) {
                hipLaunchKernelGGL((contract_lowp_resident_kernel<NB, MB, FP16, SR, SB, true, true>), dim3(n_wg),
                                   dim3(512), resident_bytes, s, a, frag, k, g.n_rg, g.n_q, g.lds_pitch,
                                   g.lds_rows, tiles_x, n_tiles, per, xs);
                return hip_status(hipGetLastError(), "contract_lowp_resident_kernel");
            }
        }
        if (reg)
            hipLaunchKernelGGL((contract_lowp_resident_kernel<NB, MB, FP16, SR, SB, true, false>), dim3(n_wg),
                               dim3(512), resident_bytes, s, a, frag, k, g.n_rg, g.n_q, g.lds_pitch,
                               g.lds_rows, tiles_x, n_tiles, per, xs);
        else
            hipLaunchKernelGGL((contract_lowp_resident_kernel<NB, MB, FP16, SR, SB, false, false>), dim3(n_wg),
                               dim3(512), resident_bytes, s, a, frag, k, g.n_rg, g.n_q, g.lds_pitch,
                               g.lds_rows, tiles_x, n_tiles, per, xs);
        return hip_status(hipGetLastError(), "contract_lowp_resident_kernel");
    }
    if (reg)
        hipLaunchKernelGGL((contract_lowp_kernel<NB, MB, FP16, SR, SB, true>), dim3(n_tiles), dim3(512),
                           g.lds_bytes, s, a, frag, k, g.n_rg, g.n_q, g.lds_pitch, g.lds_rows,
                           tiles_x, n_tiles, xs);
    else
        hipLaunchKernelGGL((contract_lowp_kernel<NB, MB, FP16, SR, SB, false>), dim3(n_tiles),
                           dim3(512), g.lds_bytes, s, a, frag, k, g.n_rg, g.n_q, g.lds_pitch,
                           g.lds_rows, tiles_x, n_tiles, xs);
    return hip_status(hipGetLastError(), "contract_lowp_kernel");
}

template <int MB, bool FP16, bool SR, bool SB>
static int launch_lowp_nbm(const ContractArgs& a, const uint16_t* frag, int nb, bool reg,
                           hipStream_t s) {
    switch (nb) {
        case 1: return launch_lowp_t<1, MB, FP16, SR, SB>(a, frag, reg, s);
        case 2: return launch_lowp_t<2, MB, FP16, SR, SB>(a, frag, reg, s);
        case 3: return launch_lowp_t<3, MB, FP16, SR, SB>(a, frag, reg, s);
        case 4:
            // 49+ filters with more than 16 spatial terms exceed N * M <= 1024
            if constexpr (MB == 1) return launch_lowp_t<4, MB, FP16, SR, SB>(a, frag, reg, s);
            return fail(SVCONV_EUNSUPPORTED, "more than 48 filters with more than 16 terms");
        default: return fail(SVCONV_EUNSUPPORTED, "more than 64 filters");
    }
}

template <bool FP16, bool SR, bool SB>
static int launch_lowp_nb(const ContractArgs& a, const uint16_t* frag, int nb, bool reg,
                          hipStream_t s) {
    if (a.M <= 16) return launch_lowp_nbm<1, FP16, SR, SB>(a, frag, nb, reg, s);
    return launch_lowp_nbm<2, FP16, SR, SB>(a, frag, nb, reg, s);
}

int launch_contract_lowp(const ContractArgs& a, const uint16_t* frag, int nb, int precision,
                         hipStream_t s) {
    const int k = 2 * a.h + 1;
    if (k > 8 * LP_NQ)
        return fail(SVCONV_EUNSUPPORTED, "bf16/fp16 forms support half-widths up to 15");
    const bool reg = (a.coef == nullptr);
    switch (precision) {
        case SVCONV_BF16: return launch_lowp_nb<false, false, false>(a, frag, nb, reg, s);
        case SVCONV_FP16: return launch_lowp_nb<true, false, false>(a, frag, nb, reg, s);
        case SVCONV_BF16X3: return launch_lowp_nb<false, true, true>(a, frag, nb, reg, s);
        case SVCONV_FP16X2: return launch_lowp_nb<true, true, false>(a, frag, nb, reg, s);
        case SVCONV_FP16X3: return launch_lowp_nb<true, true, true>(a, frag, nb, reg, s);
        default: return fail(SVCONV_EINVAL, "not a low-precision form");
    }
}

}  // namespace svc
