// Separable form of the Gaussian-basis contraction.
//
// Every Gaussian basis function is a product of two one-dimensional factors
// (Sec. 2, Eq. 2 with the Gaussian basis of Alard & Lupton):
//   B_n(u,v) = exp(-(u^2+v^2)/(2 s^2)) u^i v^j / Z = f_i(u) f_j(v),
//   f_e(w) = exp(-w^2/(2 s^2)) w^e / sum_w |exp(-w^2/(2 s^2)) w^e|,
// because the L1 norm of the product is the product of the two L1 norms.  So
//   T_n = B_n (x) R = f_j (x)_y ( f_i (x)_x R ),
// a row pass with the (d+1) factors f_i of a Gaussian family followed by a
// column pass with f_j on each row response: (d+1) + N one-dimensional
// convolutions of k taps per pixel instead of N two-dimensional ones of k^2.
// The result is D of Eq. 1 exactly, up to rounding.
//
// Arithmetic: float64 fused multiply-adds on the vector units (on this chip
// the float64 vector rate equals the unpacked float32 rate); the row
// responses are rounded to float32 once, in LDS, between the two passes.  The
// pedestal s is subtracted from R when it is staged and restored through
// s * beta_n, as in the matrix-core forms.
//
// Both passes use the symmetry of the factors (f_e is even or odd in w with
// e): each pair of taps +-w costs one add, shared by all factors of a parity,
// and one FMA per factor (fold_conv below).
//
// Workgroup: SEP_NW waves, output tile 64 x (RPT SEP_NW) with RPT = SEP_ROWS
// rows per thread (half as many in the T-only instances of kernels wider than
// 21 taps, sep_rpt).  Phase A (row pass): each task is one staged row and
// SEP_AOUT consecutive columns, computing up to SEP_CHUNK row factors from one
// register window.  Phase B (column pass): thread (lane x, wave w) owns
// column x and RPT rows; it
// reads the column of a row response into registers once and applies every
// column factor of that row factor, four at a time, then folds T_n + s beta_n
// into D with c_n(x,y) = sum_m a_nm P_m.
#include "internal.hpp"
#include "sep_fold.hpp"

namespace svc {

#ifndef SEP_WAVES
#define SEP_WAVES 8
#endif
#ifndef SEP_ROWS
#define SEP_ROWS 8
#endif
#ifndef SEP_AOUT
#define SEP_AOUT 8
#endif
constexpr int SEP_NW = SEP_WAVES;          // waves per workgroup
constexpr int SEP_RPT = SEP_ROWS;          // output rows per thread (phase B)
constexpr int SEP_APT = SEP_AOUT;          // row-pass outputs per task (phase A)
constexpr int SEP_TW = 64;
// Rows per thread of an instance: the T-only instances of wide kernels take
// half as many, because their basis-response stores and folded column
// factors would not fit the registers of SEP_RPT rows without spilling.
constexpr int sep_rpt(int h, bool tonly) { return (tonly && h > 10) ? SEP_RPT / 2 : SEP_RPT; }
#ifndef SEP_ROUND
#define SEP_ROUND 4
#endif
constexpr int SEP_CHUNK = SEP_ROUND;       // row factors per phase A / phase B round
// rounds start at even factors (the fold needs the parity of each factor) and
// a round folds at most 4 factors together
static_assert(SEP_CHUNK == 2 || SEP_CHUNK == 4, "SEP_ROUND must be 2 or 4");

// One basis response T_n on a thread's RPT rows: in the T-only mode
// written out as T_n + s beta_n, else D += c_n T_n with
// c_n(x, y) = sum_q Cy[q] yh^q (Horner in yh; DSM bounds the spatial degree
// of the kernel instance).  The pedestal term s beta_n c_n is summed once per
// pixel at the end.
template <bool TONLY, int DSM, int RPT>
__device__ __forceinline__ void sep_basis_out(const SepArgs& a, int n, const double (&tv)[RPT],
                                              int x, int y0, int y_end, int d_s,
                                              const double (&xpow)[DSM + 1],
                                              const double (&yh)[RPT], double (&dacc)[RPT]) {
    if (TONLY) {
        const double pbt = (double)a.ped * as_const(a.beta)[n];
        if (x < a.W) {
#pragma unroll
            for (int o = 0; o < RPT; ++o) {
                const int y = y0 + o;
                if (y < y_end) a.tout[((size_t)n * a.n_rows + (y - a.y_begin)) * a.W + x] = (float)(tv[o] + pbt);
            }
        }
        return;
    }
    double cy[DSM + 1];
    coef_in_x<DSM>(as_const(a.coefp) + (size_t)n * kSepCoefPad, xpow, cy);
#pragma unroll
    for (int o = 0; o < RPT; ++o) {
        double cn = cy[DSM];
#pragma unroll
        for (int q = DSM - 1; q >= 0; --q) cn = fma(cn, yh[o], cy[q]);
        dacc[o] = fma(cn, tv[o], dacc[o]);
    }
}

template <int H, bool TONLY, int DSM>
__global__ __launch_bounds__(64 * SEP_NW) void contract_sep_kernel(SepArgs a) {
    constexpr int NT = 64 * SEP_NW;
    constexpr int RPT = sep_rpt(H, TONLY);     // output rows per thread
    constexpr int TH = RPT * SEP_NW;            // output rows per tile
    constexpr int K = 2 * H + 1;
    constexpr int RA = TH + 2 * H;              // staged rows
    constexpr int CA = SEP_TW + 2 * H;          // staged columns
    constexpr int TP = CA | 1;                  // tile pitch (floats), odd: rows hit distinct banks
    constexpr int RP = SEP_TW + 1;              // row-response pitch, odd for the same reason
    constexpr int WA = SEP_APT + 2 * H;         // phase-A window
    constexpr int WB = RPT + 2 * H;             // phase-B window
    constexpr int NTASK = RA * (SEP_TW / SEP_APT);
    extern __shared__ float sep_lds[];
    float* tile = sep_lds;                      // [RA][TP]
    float* rc = sep_lds + RA * TP;              // [SEP_CHUNK][RA][RP]

    const cptr<double> f1d = as_const(a.f1d);
    const cptr<int> fam = as_const(a.fam);

    const int tid = threadIdx.x;
    const int t = sep_xcd_remap(blockIdx.x, a.n_tiles);
    const int X0 = (t % a.tiles_x) * SEP_TW;
    const int Y0 = a.y_begin + (t / a.tiles_x) * TH;
    const int y_end = min(a.H, a.y_begin + a.n_rows);

    // stage R - s; outside the image R is 0, so the staged value is -s there.
    // The loads of SEP_SB elements per thread are issued together from
    // clamped addresses and the masks apply when storing, so that a batch
    // waits for memory once.
    constexpr int SEP_SB = 8;
    for (int q0 = tid; q0 < RA * CA; q0 += NT * SEP_SB) {
        float v[SEP_SB];
#pragma unroll
        for (int sb = 0; sb < SEP_SB; ++sb) {
            const int q = q0 + NT * sb;
            const int r = q / CA, c = q - r * CA;
            const int gy = Y0 - H + r, gx = X0 - H + c;
            v[sb] = a.X[(size_t)(gy < 0 ? 0 : (gy < a.H ? gy : a.H - 1)) * a.W +
                        (gx < 0 ? 0 : (gx < a.W ? gx : a.W - 1))];
        }
#pragma unroll
        for (int sb = 0; sb < SEP_SB; ++sb) {
            const int q = q0 + NT * sb;
            const int r = q / CA, c = q - r * CA;
            const int gy = Y0 - H + r, gx = X0 - H + c;
            const bool in = gy >= 0 && gy < a.H && gx >= 0 && gx < a.W;
            if (q < RA * CA) tile[r * TP + c] = (in ? v[sb] : 0.f) - a.ped;
        }
    }

    const int lane = tid & 63, w = tid >> 6;
    const int x = X0 + lane;
    const double xh = a.sx * x + a.ox;
    double xpow[DSM + 1];
    xpow[0] = 1.0;
#pragma unroll
    for (int q = 1; q <= DSM; ++q) xpow[q] = xpow[q - 1] * xh;
    double yh[RPT], dacc[RPT];
#pragma unroll
    for (int rr = 0; rr < RPT; ++rr) {
        yh[rr] = a.sy * (Y0 + RPT * w + rr) + a.oy;
        dacc[rr] = 0.0;
    }
    const int d_s = a.d_s;

    for (int g = 0; g < a.G; ++g) {
        const int deg = fam[2 * g], base = fam[2 * g + 1];
        const cptr<double> fg = f1d + (size_t)g * kSepMaxFactors * K;
        for (int i0 = 0; i0 <= deg; i0 += SEP_CHUNK) {
            const int nc = min(SEP_CHUNK, deg + 1 - i0);
            __syncthreads();   // tile staged / previous round's rc consumed
            // phase A: rc[c][r][x'] = sum_u f_{i0+c}(u) (R - s)(x' - u, r)
            for (int tb = 0; tb < NTASK; tb += NT) {
                const int task = tb + tid;
                if (task < NTASK) {
                    // consecutive lanes take consecutive rows (odd pitches: no bank conflicts)
                    const int qi = task / RA, r = task - qi * RA;
                    const int q4 = SEP_APT * qi;
                    double win[WA];
#pragma unroll
                    for (int s = 0; s < WA; ++s) win[s] = (double)tile[r * TP + q4 + s];
                    // the round's factors i0..i0+nc-1 as an even and an odd group
                    auto group = [&](auto odd_c) {
                        constexpr int par = decltype(odd_c)::value ? 1 : 0;
                        const int nf = (nc - par + 1) / 2;
                        if (nf > 0) {
                            with_nf(nf, [&](auto nf_c) {
                                constexpr int NF = decltype(nf_c)::value < 2 ? decltype(nf_c)::value : 2;
                                double acc[NF][SEP_APT];
                                fold_conv<H, NF, SEP_APT, par == 1>(win, fg + (size_t)(i0 + par) * K, acc);
#pragma unroll
                                for (int cc = 0; cc < NF; ++cc) {
                                    float* dst = rc + ((size_t)(par + 2 * cc) * RA + r) * RP + q4;
#pragma unroll
                                    for (int o = 0; o < SEP_APT; ++o) dst[o] = (float)acc[cc][o];
                                }
                            });
                        }
                    };
                    group(std::false_type{});
                    group(std::true_type{});
                }
            }
            __syncthreads();
            // phase B: T_n(x, y) = sum_v f_j(v) rc(x, y - v), D += c_n (T_n + s beta_n)
            for (int c = 0; c < nc; ++c) {
                const int i = i0 + c;
                double col[WB];
#pragma unroll
                for (int s = 0; s < WB; ++s) col[s] = (double)rc[((size_t)c * RA + RPT * w + s) * RP + lane];
                // the column factors of row factor i in two groups of one
                // parity, f_0, f_2, ... and f_1, f_3, ..., up to 4 folded together
                // (a degree above 7 leaves f_8 or f_9, applied unfolded)
                auto group = [&](auto odd_c) {
                    constexpr int par = decltype(odd_c)::value ? 1 : 0;
                    if (deg - i < par) return;
                    const int cnt = (deg - i - par) / 2 + 1;   // j = par, par + 2, ... <= deg - i
                    const int nf = min(cnt, 4);
                    with_nf(nf, [&](auto nf_c) {
                        constexpr int NF = decltype(nf_c)::value;
                        double tv[NF][RPT];
                        fold_conv<H, NF, RPT, par == 1>(col, fg + (size_t)par * K, tv);
#pragma unroll
                        for (int jj = 0; jj < NF; ++jj) {
                            const int j = par + 2 * jj;
                            sep_basis_out<TONLY, DSM, RPT>(a, base + (i + j) * (i + j + 1) / 2 + j, tv[jj], x,
                                                      Y0 + RPT * w, y_end, d_s, xpow, yh, dacc);
                        }
                    });
                    if (cnt > 4) {
                        const int j = par + 8;
                        double tv1[RPT];
                        direct_conv<H, RPT>(col, fg + (size_t)j * K, tv1);
                        sep_basis_out<TONLY, DSM, RPT>(a, base + (i + j) * (i + j + 1) / 2 + j, tv1, x,
                                              Y0 + RPT * w, y_end, d_s, xpow, yh, dacc);
                    }
                };
                group(std::false_type{});
                group(std::true_type{});
            }
        }
    }
    if (!TONLY && x < a.W) {
        // I of the thread's rows, requested together from clamped rows (X
        // stands in when there is no I; unused values are never read)
        float ivr[RPT];
        const float* ip = a.I ? a.I : a.X;
#pragma unroll
        for (int o = 0; o < RPT; ++o) {
            const int y = Y0 + RPT * w + o;
            ivr[o] = ip[(size_t)(y < y_end ? y : y_end - 1) * a.W + x];
        }
        // pedestal restore: s sum_n beta_n c_n = s sum_m gamma_m P_m
        double cy[DSM + 1];
        coef_in_x<DSM>(as_const(a.gammap), xpow, cy);
#pragma unroll
        for (int o = 0; o < RPT; ++o) {
            const int y = Y0 + RPT * w + o;
            if (y < y_end) {
                double pg = cy[DSM];
#pragma unroll
                for (int q = DSM - 1; q >= 0; --q) pg = fma(pg, yh[o], cy[q]);
                const size_t idx = (size_t)y * a.W + x;
                const double iv = a.I ? (double)ivr[o] : 0.0;
                a.out[idx] = (float)(fma((double)a.ped, pg, dacc[o]) - iv);
            }
        }
    }
}

// Per-call tables of the separable epilogue: coef in float64 (read by scalar
// loads without conversions), gamma_m = sum_n coef[n][m] beta_n, and, when
// coefp is given, both again with the stride kSepCoefPad and zeros beyond M
// (coefp[N * kSepCoefPad + m] is gamma), so that the contraction reads a
// fixed number of terms without branches, followed by a float32 copy of the
// coefficients in the same layout (N + 1 rows, the last one zero).
__global__ __launch_bounds__(1024) void sep_prep_kernel(const float* __restrict__ coef,
                                                        const double* __restrict__ beta, int N,
                                                        int M, double* __restrict__ coefd,
                                                        double* __restrict__ gamma,
                                                        double* __restrict__ coefp) {
    for (int i = threadIdx.x; i < N * M; i += 1024) coefd[i] = (double)coef[i];
    if (coefp) {
        float* coefpf = reinterpret_cast<float*>(coefp + (size_t)(N + 1) * kSepCoefPad);
        for (int i = threadIdx.x; i < (N + 1) * kSepCoefPad; i += 1024) {
            const int n = i / kSepCoefPad, m = i - n * kSepCoefPad;
            const float c = (n < N && m < M) ? coef[n * M + m] : 0.f;
            if (n < N) coefp[i] = (double)c;
            coefpf[i] = c;
        }
    }
    // gamma_m: one wave per term, the lanes over the bases, summed across the wave
    const int wave = threadIdx.x >> 6, ln = threadIdx.x & 63;
    for (int m = wave; m < kSepCoefPad; m += 1024 / 64) {
        double v = 0.0;
        if (m < M)
            for (int n = ln; n < N; n += 64) v = fma((double)coef[n * M + m], beta[n], v);
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
        if (ln == 0) {
            if (m < M) gamma[m] = v;
            if (coefp) coefp[(size_t)N * kSepCoefPad + m] = v;
        }
    }
}

int launch_sep_prep(const float* coef, const double* beta, int N, int M, double* coefd,
                    double* gamma, double* coefp, hipStream_t s) {
    hipLaunchKernelGGL(sep_prep_kernel, dim3(1), dim3(1024), 0, s, coef, beta, N, M, coefd, gamma, coefp);
    return hip_status(hipGetLastError(), "sep_prep_kernel");
}

template <int H, bool TONLY, int DSM>
static int launch_sep_i(SepArgs a, hipStream_t s) {
    constexpr int TH = sep_rpt(H, TONLY) * SEP_NW;
    constexpr int RA = TH + 2 * H, CA = SEP_TW + 2 * H;
    const size_t lds = ((size_t)RA * (CA | 1) + (size_t)SEP_CHUNK * RA * (SEP_TW + 1)) * sizeof(float);
    a.tiles_x = (a.W + SEP_TW - 1) / SEP_TW;
    a.n_tiles = a.tiles_x * ((a.n_rows + TH - 1) / TH);
    hipLaunchKernelGGL((contract_sep_kernel<H, TONLY, DSM>), dim3(a.n_tiles), dim3(64 * SEP_NW), lds, s, a);
    return hip_status(hipGetLastError(), "contract_sep_kernel");
}

template <int H>
static int launch_sep_t(const SepArgs& a, hipStream_t s) {
    // TONLY: write the basis responses T_n + s beta_n instead of D; spatial
    // degrees up to 2 take the instance with the short polynomial in yh
    if (a.tout) return launch_sep_i<H, true, 0>(a, s);
    if (a.d_s <= 2) return launch_sep_i<H, false, 2>(a, s);
    return launch_sep_i<H, false, kMaxSpatialDegree>(a, s);
}

int launch_contract_sep(SepArgs a, hipStream_t s) {
    switch (a.h) {
        case 1: return launch_sep_t<1>(a, s);
        case 2: return launch_sep_t<2>(a, s);
        case 3: return launch_sep_t<3>(a, s);
        case 4: return launch_sep_t<4>(a, s);
        case 5: return launch_sep_t<5>(a, s);
        case 6: return launch_sep_t<6>(a, s);
        case 7: return launch_sep_t<7>(a, s);
        case 8: return launch_sep_t<8>(a, s);
        case 9: return launch_sep_t<9>(a, s);
        case 10: return launch_sep_t<10>(a, s);
        case 11: return launch_sep_t<11>(a, s);
        case 12: return launch_sep_t<12>(a, s);
        case 13: return launch_sep_t<13>(a, s);
        case 14: return launch_sep_t<14>(a, s);
        case 15: return launch_sep_t<15>(a, s);
        default: return fail(SVCONV_EUNSUPPORTED, "separable form needs 1 <= half-width <= 15");
    }
}

}  // namespace svc
