// Adjoint in the coefficients through the separable Gaussian factors.
//
//   dL/da[n][m] = sum_p G(p) P_m(p) T_n(p),   T_n = f_j (x)_y (f_i (x)_x R)
//
// (the factorisation of the separable forward form).  With the pedestal s,
// T_n(R) = T_n(R - s) + s beta_n, so
//   dL/da[n][m] = sum_p G P_m T_n(R - s) + s beta_n sum_p G P_m.
// Both sums are computed here: gP[m] = sum_p G P_m is the same moment sum
// with a response of 1, accumulated once (in the first round) in one extra
// slot, and the final kernel adds s beta_n gP[m].
//
// A workgroup walks a 64-column strip of the image (a run of 32-row tiles).
// Rounds of SA_CHUNK row factors: the strip is walked once per round.
// Because P_m(x, y) = xh^ie yh^je and every lane keeps its column x over the
// whole walk, each lane accumulates, for the bases of one round of row
// factors, the moments V[n][je][lane] = sum_y G T_n yh^je (float64 LDS
// atomic adds from the 8 waves that share a column); the weighting by xh^ie
// and the sum over the 64 columns happen once per round at the end of the
// walk.  Per-workgroup results go to a partial array that a second kernel
// sums in a fixed order.
#include "internal.hpp"
#include "sep_fold.hpp"

namespace svc {

#ifndef SA_ROWS
#define SA_ROWS 4
#endif
#ifndef SA_ROUND
#define SA_ROUND 4
#endif
constexpr int SA_NW = 8, SA_RPT = SA_ROWS, SA_TW = 64, SA_TH = SA_NW * SA_RPT, SA_APT = 8;
constexpr int SA_CHUNK = SA_ROUND;         // row factors per round
static_assert(SA_CHUNK == 2 || SA_CHUNK == 4, "SA_ROUND must be 2 or 4 (rounds start at even factors)");

struct SepAdjArgs {
    const float* R;
    const float* G;
    int H, W;
    float ped;
    int G_fam;                  // Gaussian families
    const int* fam;             // [2 G]: degree, first basis
    const double* f1d;          // [G][kSepMaxFactors][k]
    int N, M, d_s;
    double sx, ox, sy, oy;
    int strips, tiles_y, tiles_per_seg;
    int vmax;                   // bases per round, at most
    double* part;               // [n_wg][N M]
};

// V[slot][q][lane] += sum_o G T yh^q over a thread's SA_RPT rows, q <= d_s
// (float64 LDS atomics: the 8 waves of a workgroup share a column).  The
// loop over q runs to the plan's degree; each step multiplies the row terms
// by yh once.
__device__ __forceinline__ void sa_moments(double* V, int slot, int DS1, int lane,
                                           const double (&gv)[SA_RPT], const double (&yv)[SA_RPT],
                                           const double (&tv)[SA_RPT]) {
    double t[SA_RPT];
#pragma unroll
    for (int o = 0; o < SA_RPT; ++o) t[o] = gv[o] * tv[o];
    double* vrow = V + (size_t)slot * DS1 * 64 + lane;
#pragma unroll 1
    for (int q = 0; q < DS1; ++q) {
        double m = t[0];
#pragma unroll
        for (int o = 1; o < SA_RPT; ++o) m += t[o];
        atomicAdd(vrow + q * 64, m);
#pragma unroll
        for (int o = 0; o < SA_RPT; ++o) t[o] *= yv[o];
    }
}

template <int H>
__global__ __launch_bounds__(64 * SA_NW) void adjoint_a_sep_kernel(SepAdjArgs a) {
    constexpr int NT = 64 * SA_NW;
    constexpr int K = 2 * H + 1;
    constexpr int RA = SA_TH + 2 * H, CA = SA_TW + 2 * H;
    constexpr int TP = CA | 1, RP = SA_TW + 1;
    constexpr int WA = SA_APT + 2 * H, WB = SA_RPT + 2 * H;
    constexpr int NTASK = RA * (SA_TW / SA_APT);
    const int DS1 = a.d_s + 1;
    extern __shared__ double sa_lds[];
    double* V = sa_lds;                                  // [vmax + 1][DS1][64]
    double* xpt = V + (size_t)(a.vmax + 1) * DS1 * 64;   // [DS1][64] powers of xh
    float* tile = reinterpret_cast<float*>(xpt + (size_t)DS1 * 64);   // [RA][TP]
    float* rc = tile + RA * TP;                          // [SA_CHUNK][RA][RP]

    const cptr<double> f1d = (cptr<double>)a.f1d;
    const cptr<int> fam = (cptr<int>)a.fam;

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int sxi = blockIdx.x % a.strips, seg = blockIdx.x / a.strips;
    const int X0 = sxi * SA_TW;
    const int ty0 = seg * a.tiles_per_seg;
    const int ty1 = min(a.tiles_y, ty0 + a.tiles_per_seg);
    const int x = X0 + lane;
    const int NM = a.N * a.M;
    double* part = a.part + (size_t)blockIdx.x * (NM + a.M);   // [N][M] then gP[M]

    if (w == 0) {
        const double xh = a.sx * x + a.ox;
        double pw = 1.0;
        for (int q = 0; q < DS1; ++q) {
            xpt[q * 64 + lane] = pw;
            pw *= xh;
        }
    }

    for (int g = 0; g < a.G_fam; ++g) {
        const int deg = fam[2 * g], base = fam[2 * g + 1];
        const cptr<double> fg = f1d + (size_t)g * kSepMaxFactors * K;
        for (int i0 = 0; i0 <= deg; i0 += SA_CHUNK) {
            const int nc = min(SA_CHUNK, deg + 1 - i0);
            int nn = 0;
            for (int c = 0; c < nc; ++c) nn += deg - (i0 + c) + 1;
            const bool first = (g == 0 && i0 == 0);   // this round also sums G P_m (slot nn)
            const int slots = nn + (first ? 1 : 0);
            __syncthreads();   // previous round's reduction has read V
            for (int q = tid; q < slots * DS1 * 64; q += NT) V[q] = 0.0;
            for (int ty = ty0; ty < ty1; ++ty) {
                const int Y0 = ty * SA_TH;
                __syncthreads();   // V cleared / previous tile's rc consumed
                // stage R - s: the loads of SA_SB elements per thread go out
                // together from clamped addresses, the masks apply at the store
                constexpr int SA_SB = 8;
                for (int q0 = tid; q0 < RA * CA; q0 += NT * SA_SB) {
                    float v[SA_SB];
#pragma unroll
                    for (int sb = 0; sb < SA_SB; ++sb) {
                        const int q = q0 + NT * sb;
                        const int r = q / CA, c = q - r * CA;
                        const int gy = Y0 - H + r, gx = X0 - H + c;
                        v[sb] = a.R[(size_t)(gy < 0 ? 0 : (gy < a.H ? gy : a.H - 1)) * a.W +
                                    (gx < 0 ? 0 : (gx < a.W ? gx : a.W - 1))];
                    }
#pragma unroll
                    for (int sb = 0; sb < SA_SB; ++sb) {
                        const int q = q0 + NT * sb;
                        const int r = q / CA, c = q - r * CA;
                        const int gy = Y0 - H + r, gx = X0 - H + c;
                        const bool in = gy >= 0 && gy < a.H && gx >= 0 && gx < a.W;
                        if (q < RA * CA) tile[r * TP + c] = (in ? v[sb] : 0.f) - a.ped;
                    }
                }
                __syncthreads();
                // row pass (as in the forward)
                for (int tb = 0; tb < NTASK; tb += NT) {
                    const int task = tb + tid;
                    if (task < NTASK) {
                        const int qi = task / RA, r = task - qi * RA;
                        const int q0 = SA_APT * qi;
                        double win[WA];
#pragma unroll
                        for (int s = 0; s < WA; ++s) win[s] = (double)tile[r * TP + q0 + s];
                        // the round's factors as an even and an odd group (symmetric fold)
                        auto group = [&](auto odd_c) {
                            constexpr int par = decltype(odd_c)::value ? 1 : 0;
                            const int nf = (nc - par + 1) / 2;
                            if (nf > 0) {
                                with_nf(nf, [&](auto nf_c) {
                                    constexpr int NF = decltype(nf_c)::value < 2 ? decltype(nf_c)::value : 2;
                                    double acc[NF][SA_APT];
                                    fold_conv<H, NF, SA_APT, par == 1>(win, fg + (size_t)(i0 + par) * K, acc);
#pragma unroll
                                    for (int cc = 0; cc < NF; ++cc) {
                                        float* dst = rc + ((size_t)(par + 2 * cc) * RA + r) * RP + q0;
#pragma unroll
                                        for (int o = 0; o < SA_APT; ++o) dst[o] = (float)acc[cc][o];
                                    }
                                });
                            }
                        };
                        group(std::false_type{});
                        group(std::true_type{});
                    }
                }
                __syncthreads();
                // column pass per basis, moments of G T_n over this thread's rows
                double gv[SA_RPT], yv[SA_RPT];
                {
                    // requested together from clamped addresses, masked after
                    float gr[SA_RPT];
                    const int xc = x < a.W ? x : a.W - 1;
#pragma unroll
                    for (int o = 0; o < SA_RPT; ++o) {
                        const int y = Y0 + SA_RPT * w + o;
                        gr[o] = a.G[(size_t)(y < a.H ? y : a.H - 1) * a.W + xc];
                    }
#pragma unroll
                    for (int o = 0; o < SA_RPT; ++o) {
                        const int y = Y0 + SA_RPT * w + o;
                        gv[o] = (x < a.W && y < a.H) ? (double)gr[o] : 0.0;
                        yv[o] = a.sy * y + a.oy;
                    }
                }
                if (first) {
                    double ones[SA_RPT];
#pragma unroll
                    for (int o = 0; o < SA_RPT; ++o) ones[o] = 1.0;
                    sa_moments(V, nn, DS1, lane, gv, yv, ones);   // G P_m sums
                }
                int nl = 0;   // slot of basis (i, 0) in this round
                for (int c = 0; c < nc; ++c) {
                    const int i = i0 + c;
                    double col[WB];
#pragma unroll
                    for (int s = 0; s < WB; ++s) col[s] = (double)rc[((size_t)c * RA + SA_RPT * w + s) * RP + lane];
                    // column factors f_0, f_2, ... and f_1, f_3, ... of row factor i, folded
                    auto group = [&](auto odd_c) {
                        constexpr int par = decltype(odd_c)::value ? 1 : 0;
                        if (deg - i < par) return;
                        const int cnt = (deg - i - par) / 2 + 1;
                        with_nf(min(cnt, 4), [&](auto nf_c) {
                            constexpr int NF = decltype(nf_c)::value;
                            double tv[NF][SA_RPT];
                            fold_conv<H, NF, SA_RPT, par == 1>(col, fg + (size_t)par * K, tv);
#pragma unroll
                            for (int jj = 0; jj < NF; ++jj) sa_moments(V, nl + par + 2 * jj, DS1, lane, gv, yv, tv[jj]);
                        });
                        if (cnt > 4) {
                            double tv1[SA_RPT];
                            direct_conv<H, SA_RPT>(col, fg + (size_t)(par + 8) * K, tv1);
                            sa_moments(V, nl + par + 8, DS1, lane, gv, yv, tv1);
                        }
                    };
                    group(std::false_type{});
                    group(std::true_type{});
                    nl += deg - i + 1;
                }
            }
            __syncthreads();
            // dL/da[n][m] (this strip) = sum_lanes xh^ie V[n][je][lane]
            for (int q = tid; q < slots * a.M; q += NT) {
                int l = q / a.M;
                const int m = q - l * a.M;
                int t = 0;
                while ((t + 1) * (t + 2) / 2 <= m) ++t;
                const int je = m - t * (t + 1) / 2, ie = t - je;
                int n = a.N;                     // slot nn: the G P_m sums
                for (int c = 0; c < nc && n == a.N && l < nn; ++c) {
                    const int cnt = deg - (i0 + c) + 1;
                    if (l < cnt) n = base + (i0 + c + l) * (i0 + c + l + 1) / 2 + l;
                    else l -= cnt;
                }
                const int vl = q / a.M;
                double s = 0.0;
                for (int ln = 0; ln < 64; ++ln)
                    s = fma(xpt[ie * 64 + ln], V[((size_t)vl * DS1 + je) * 64 + ln], s);
                part[(size_t)n * a.M + m] = s;
            }
        }
    }
}

// ga[n][m] = sum over workgroups (fixed order) + s beta_n gP[m]
__global__ void adjoint_a_sep_final(const double* __restrict__ part, int n_wg, int N, int M,
                                    const double* __restrict__ beta, float ped,
                                    double* __restrict__ ga) {
    const int nm = blockIdx.x * blockDim.x + threadIdx.x;
    if (nm >= N * M) return;
    const int n = nm / M, m = nm - n * M;
    const size_t stride = (size_t)(N + 1) * M;
    double s = 0.0, gp = 0.0;
    for (int b = 0; b < n_wg; ++b) {
        s += part[b * stride + nm];
        gp += part[b * stride + (size_t)N * M + m];
    }
    ga[nm] = s + (double)ped * beta[n] * gp;
}

template <int H>
static int launch_asep_t(const SepAdjArgs& a, int n_wg, size_t lds, hipStream_t s) {
    hipLaunchKernelGGL(adjoint_a_sep_kernel<H>, dim3(n_wg), dim3(64 * SA_NW), lds, s, a);
    return hip_status(hipGetLastError(), "adjoint_a_sep_kernel");
}

static int sep_round_bases(const svconv_plan* p) {
    int vmax = 0;                              // bases in one round of row factors, at most
    for (int d : p->degrees)
        for (int i0 = 0; i0 <= d; i0 += SA_CHUNK) {
            int nn = 0;
            for (int c = 0; c < SA_CHUNK && i0 + c <= d; ++c) nn += d - (i0 + c) + 1;
            vmax = nn > vmax ? nn : vmax;
        }
    return vmax;
}

static size_t sep_adjoint_lds(const svconv_plan* p) {
    const int RA = SA_TH + 2 * p->h, CA = SA_TW + 2 * p->h;
    return ((size_t)(sep_round_bases(p) + 1) * (p->d_s + 1) * 64 + (size_t)(p->d_s + 1) * 64) *
               sizeof(double) +
           ((size_t)RA * (CA | 1) + (size_t)SA_CHUNK * RA * (SA_TW + 1)) * sizeof(float);
}

bool sep_adjoint_supported(const svconv_plan* p) {
    return p->dSep1d && p->h >= 1 && p->h <= 15 && sep_adjoint_lds(p) <= 160 * 1024;
}

int launch_adjoint_a_sep(svconv_plan* p, const float* R, const float* G, double* ga) {
    if (!sep_adjoint_supported(p))
        return fail(SVCONV_EUNSUPPORTED, "separable adjoint: Gaussian bases, 1 <= half-width <= 15 and its LDS budget");
    const int h = p->h, NM = p->N * p->M;
    SepAdjArgs a{};
    a.R = R;
    a.G = G;
    a.H = p->H;
    a.W = p->W;
    a.ped = p->pedestal;
    a.G_fam = (int)p->sigmas.size();
    a.fam = p->dSepFam;
    a.f1d = p->dSep1d;
    a.N = p->N;
    a.M = p->M;
    a.d_s = p->d_s;
    if (p->Wf > 1) { a.sx = 2.0 / (p->Wf - 1); a.ox = a.sx * p->x0 - 1.0; }
    if (p->Hf > 1) { a.sy = 2.0 / (p->Hf - 1); a.oy = a.sy * p->y0 - 1.0; }
    a.vmax = sep_round_bases(p);
    a.strips = (p->W + SA_TW - 1) / SA_TW;
    a.tiles_y = (p->H + SA_TH - 1) / SA_TH;
    // about two workgroups per CU, within the partial-sum scratch
    const size_t cap = adjoint_scratch_doubles(p->H, p->W, p->k, p->M) / (size_t)(NM + p->M) - 1;
    int segs = (512 + a.strips - 1) / a.strips;
    if (segs > a.tiles_y) segs = a.tiles_y;
    a.tiles_per_seg = (a.tiles_y + segs - 1) / segs;
    segs = (a.tiles_y + a.tiles_per_seg - 1) / a.tiles_per_seg;
    while ((size_t)a.strips * segs > cap && a.tiles_per_seg < a.tiles_y) {
        a.tiles_per_seg *= 2;
        segs = (a.tiles_y + a.tiles_per_seg - 1) / a.tiles_per_seg;
    }
    const int n_wg = a.strips * segs;
    if ((size_t)n_wg > cap) return fail(SVCONV_EUNSUPPORTED, "image too wide for the adjoint scratch");
    a.part = p->dQpart;
    int st = SVCONV_OK;
    const size_t lds = sep_adjoint_lds(p);
    switch (h) {
        case 1: st = launch_asep_t<1>(a, n_wg, lds, p->stream); break;
        case 2: st = launch_asep_t<2>(a, n_wg, lds, p->stream); break;
        case 3: st = launch_asep_t<3>(a, n_wg, lds, p->stream); break;
        case 4: st = launch_asep_t<4>(a, n_wg, lds, p->stream); break;
        case 5: st = launch_asep_t<5>(a, n_wg, lds, p->stream); break;
        case 6: st = launch_asep_t<6>(a, n_wg, lds, p->stream); break;
        case 7: st = launch_asep_t<7>(a, n_wg, lds, p->stream); break;
        case 8: st = launch_asep_t<8>(a, n_wg, lds, p->stream); break;
        case 9: st = launch_asep_t<9>(a, n_wg, lds, p->stream); break;
        case 10: st = launch_asep_t<10>(a, n_wg, lds, p->stream); break;
        case 11: st = launch_asep_t<11>(a, n_wg, lds, p->stream); break;
        case 12: st = launch_asep_t<12>(a, n_wg, lds, p->stream); break;
        case 13: st = launch_asep_t<13>(a, n_wg, lds, p->stream); break;
        case 14: st = launch_asep_t<14>(a, n_wg, lds, p->stream); break;
        default: st = launch_asep_t<15>(a, n_wg, lds, p->stream); break;
    }
    if (st) return st;
    hipLaunchKernelGGL(adjoint_a_sep_final, dim3((NM + 255) / 256), dim3(256), 0, p->stream, p->dQpart,
                       n_wg, p->N, p->M, p->dBeta, p->pedestal, ga);
    return hip_status(hipGetLastError(), "adjoint_a_sep_final");
}

}  // namespace svc

// ------------------------------------------------------- adjoint in R ----
//
//   dL/dR(q) = sum_n sum_{u,v} B_n[u,v] E_n(q + (u,v)),   E_n = c_n G,
//
// and with B_n = f_i(u) f_j(v) the inner sums group by row factor:
//   CE_i(x', y) = sum_j sum_v f_j(v) E_{ij}(x', y + v)       (column pass per basis)
//   dL/dR(x, y) += sum_u f_i(u) CE_i(x + u, y)              (row pass per factor).
// A workgroup owns a 64 x 64 output tile.  For every basis it forms E_n on the
// tile and its halo in LDS (c_n from per-column coefficients in xh and Horner
// in yh, G read from global memory), then column tasks (one staged column, 8 output rows) accumulate
// CE_i in registers over the bases of the row factor; CE_i goes to LDS and
// each thread adds the row pass to its 8 output pixels.  E and CE are held
// in float32 between passes, every sum in float64.

namespace svc {

constexpr int SR_NT = 512, SR_TW = 64, SR_TH = 64, SR_RPT = 8;

struct SepRArgs {
    const float* G;
    float* gR;
    int H, W;
    int G_fam;
    const int* fam;
    const double* f1d;
    const double* coefd;        // [N][M] float64 coefficients
    int M, d_s;
    double sx, ox, sy, oy;
    int tiles_x, n_tiles;
};

// G is read from global memory (L2) while E_n is formed, not staged in LDS:
// the LDS left then holds two workgroups per CU, and the register budget is
// held to 4 waves per SIMD; this was faster than an LDS copy of G at one
// workgroup per CU.
#ifndef SR_GLOBAL_G
#define SR_GLOBAL_G 1
#endif
#ifndef SR_WG_PER_CU
#define SR_WG_PER_CU 4          // minimum waves per SIMD (launch bounds)
#endif
template <int H>
__global__ __launch_bounds__(SR_NT, SR_WG_PER_CU) void adjoint_r_sep_kernel(SepRArgs a) {
    constexpr int K = 2 * H + 1;
    constexpr int RA = SR_TH + 2 * H, CA = SR_TW + 2 * H, CP = CA | 1;
    constexpr int WB = SR_RPT + 2 * H;                  // window of a column task / row task
    constexpr int NTASK = CA * (SR_TH / SR_RPT);        // column tasks
    constexpr int TPT = (NTASK + SR_NT - 1) / SR_NT;    // column tasks per thread
    constexpr int DSM = kMaxSpatialDegree + 1;
    extern __shared__ double sr_lds[];
    double* cyt = sr_lds;                               // [CA][DSM] coefficients in yh per column
    float* gt = reinterpret_cast<float*>(cyt + CA * DSM);   // [RA][CP] G tile
    float* en = gt + (SR_GLOBAL_G ? 0 : RA * CP);       // [RA][CP] E_n tile
    float* ce = en + RA * CP;                           // [SR_TH][CP] CE_i

    const cptr<double> f1d = (cptr<double>)a.f1d;
    const cptr<int> fam = (cptr<int>)a.fam;
    const cptr<double> coefd = (cptr<double>)a.coefd;
    const int tid = threadIdx.x;
    const int t = sep_xcd_remap(blockIdx.x, a.n_tiles);
    const int X0 = (t % a.tiles_x) * SR_TW, Y0 = (t / a.tiles_x) * SR_TH;
    const int DS1 = a.d_s + 1;

    if (!SR_GLOBAL_G)
        for (int q = tid; q < RA * CA; q += SR_NT) {
            const int r = q / CA, c = q - r * CA;
            const int gy = Y0 - H + r, gx = X0 - H + c;
            const float v = a.G[(size_t)(gy < 0 ? 0 : (gy < a.H ? gy : a.H - 1)) * a.W +
                                (gx < 0 ? 0 : (gx < a.W ? gx : a.W - 1))];
            gt[r * CP + c] = (gy >= 0 && gy < a.H && gx >= 0 && gx < a.W) ? v : 0.f;
        }
    // row-pass role: output row rr, columns q8 .. q8 + 7
    const int rr = tid >> 3, q8 = (tid & 7) * SR_RPT;
    double gacc[SR_RPT];
#pragma unroll
    for (int o = 0; o < SR_RPT; ++o) gacc[o] = 0.0;

    for (int g = 0; g < a.G_fam; ++g) {
        const int deg = fam[2 * g], base = fam[2 * g + 1];
        const cptr<double> fg = f1d + (size_t)g * kSepMaxFactors * K;
        for (int i = 0; i <= deg; ++i) {
            double cacc[TPT][SR_RPT];
#pragma unroll
            for (int tk = 0; tk < TPT; ++tk)
#pragma unroll
                for (int o = 0; o < SR_RPT; ++o) cacc[tk][o] = 0.0;
            for (int j = 0; j + i <= deg; ++j) {
                const int n = base + (i + j) * (i + j + 1) / 2 + j;
                const cptr<double> an = coefd + (size_t)n * a.M;
                __syncthreads();   // previous E_n / cyt consumed (and G staged)
                // coefficients of c_n in yh for every staged column
                for (int e = tid; e < CA * DS1; e += SR_NT) {
                    const int c = e / DS1, jj = e - c * DS1;
                    const double xh = a.sx * (X0 - H + c) + a.ox;
                    double s = 0.0, xp = 1.0;
                    for (int ie = 0; ie + jj <= a.d_s; ++ie) {
                        const int tt = ie + jj;
                        s = fma(an[tt * (tt + 1) / 2 + jj], xp, s);
                        xp *= xh;
                    }
                    cyt[c * DSM + jj] = s;
                }
                __syncthreads();
                // E_n = c_n G on the staged region
                for (int q = tid; q < RA * CA; q += SR_NT) {
                    const int r = q / CA, c = q - r * CA;
                    const double yh = a.sy * (Y0 - H + r) + a.oy;
                    double cn = 0.0;
                    for (int jj = a.d_s; jj >= 0; --jj) cn = fma(cn, yh, cyt[c * DSM + jj]);
                    float gv;
                    if (SR_GLOBAL_G) {
                        // clamped address, masked after (no branch around the load)
                        const int gy = Y0 - H + r, gx = X0 - H + c;
                        const float v = a.G[(size_t)(gy < 0 ? 0 : (gy < a.H ? gy : a.H - 1)) * a.W +
                                            (gx < 0 ? 0 : (gx < a.W ? gx : a.W - 1))];
                        gv = (gy >= 0 && gy < a.H && gx >= 0 && gx < a.W) ? v : 0.f;
                    } else {
                        gv = gt[r * CP + c];
                    }
                    en[r * CP + c] = (float)(cn * (double)gv);
                }
                __syncthreads();
                // column correlation with f_j, accumulated over j
                const cptr<double> f = fg + (size_t)j * K;
#pragma unroll
                for (int tk = 0; tk < TPT; ++tk) {
                    const int task = tid + tk * SR_NT;
                    if (task < NTASK) {
                        const int c = task % CA, r0 = (task / CA) * SR_RPT;
                        // the window stays in float32 and a rolling set of
                        // SR_RPT samples is widened to float64 as the taps
                        // advance, which keeps the registers of wide kernels
                        // within the occupancy target
                        float winf[WB];
#pragma unroll
                        for (int s = 0; s < WB; ++s) winf[s] = en[(r0 + s) * CP + c];
                        double roll[SR_RPT];
#pragma unroll
                        for (int o = 0; o < SR_RPT; ++o) roll[o] = (double)winf[o];
#pragma unroll
                        for (int v = 0; v < K; ++v) {
                            const double fv = f[v];
#pragma unroll
                            for (int o = 0; o < SR_RPT; ++o) cacc[tk][o] = fma(fv, roll[o], cacc[tk][o]);
                            if (v + 1 < K) {
#pragma unroll
                                for (int o = 0; o + 1 < SR_RPT; ++o) roll[o] = roll[o + 1];
                                roll[SR_RPT - 1] = (double)winf[v + SR_RPT];
                            }
                        }
                    }
                }
            }
            // CE_i to LDS, then the row correlation with f_i
#pragma unroll
            for (int tk = 0; tk < TPT; ++tk) {
                const int task = tid + tk * SR_NT;
                if (task < NTASK) {
                    const int c = task % CA, r0 = (task / CA) * SR_RPT;
#pragma unroll
                    for (int o = 0; o < SR_RPT; ++o) ce[(r0 + o) * CP + c] = (float)cacc[tk][o];
                }
            }
            __syncthreads();
            {
                const cptr<double> f = fg + (size_t)i * K;
                double win[WB];
#pragma unroll
                for (int s = 0; s < WB; ++s) win[s] = (double)ce[rr * CP + q8 + s];
#pragma unroll
                for (int u = 0; u < K; ++u) {
                    const double fu = f[u];
#pragma unroll
                    for (int o = 0; o < SR_RPT; ++o) gacc[o] = fma(fu, win[o + u], gacc[o]);
                }
            }
        }
    }
    const int y = Y0 + rr;
    if (y < a.H) {
#pragma unroll
        for (int o = 0; o < SR_RPT; ++o) {
            const int x = X0 + q8 + o;
            if (x < a.W) a.gR[(size_t)y * a.W + x] = (float)gacc[o];
        }
    }
}

template <int H>
static int launch_rsep_t(const SepRArgs& a, size_t lds, hipStream_t s) {
    hipLaunchKernelGGL(adjoint_r_sep_kernel<H>, dim3(a.n_tiles), dim3(SR_NT), lds, s, a);
    return hip_status(hipGetLastError(), "adjoint_r_sep_kernel");
}

int launch_adjoint_r_sep(svconv_plan* p, const float* a32, const float* G, float* gR) {
    if (!p->dSep1d || p->h < 1 || p->h > 15)
        return fail(SVCONV_EUNSUPPORTED, "separable adjoint needs Gaussian bases and 1 <= half-width <= 15");
    const int h = p->h;
    double* coefd = p->dVec + 7 * (size_t)kMaxCoefficients;
    double* gamma = p->dVec + 8 * (size_t)kMaxCoefficients;
    int st = launch_sep_prep(a32, p->dBeta, p->N, p->M, coefd, gamma, nullptr, p->stream);
    if (st) return st;
    SepRArgs a{};
    a.G = G;
    a.gR = gR;
    a.H = p->H;
    a.W = p->W;
    a.G_fam = (int)p->sigmas.size();
    a.fam = p->dSepFam;
    a.f1d = p->dSep1d;
    a.coefd = coefd;
    a.M = p->M;
    a.d_s = p->d_s;
    if (p->Wf > 1) { a.sx = 2.0 / (p->Wf - 1); a.ox = a.sx * p->x0 - 1.0; }
    if (p->Hf > 1) { a.sy = 2.0 / (p->Hf - 1); a.oy = a.sy * p->y0 - 1.0; }
    a.tiles_x = (p->W + SR_TW - 1) / SR_TW;
    a.n_tiles = a.tiles_x * ((p->H + SR_TH - 1) / SR_TH);
    const int RA = SR_TH + 2 * h, CA = SR_TW + 2 * h, CP = CA | 1;
    const size_t lds = (size_t)CA * (kMaxSpatialDegree + 1) * sizeof(double) +
                       ((size_t)(SR_GLOBAL_G ? 1 : 2) * RA * CP + (size_t)SR_TH * CP) * sizeof(float);
    switch (h) {
        case 1: return launch_rsep_t<1>(a, lds, p->stream);
        case 2: return launch_rsep_t<2>(a, lds, p->stream);
        case 3: return launch_rsep_t<3>(a, lds, p->stream);
        case 4: return launch_rsep_t<4>(a, lds, p->stream);
        case 5: return launch_rsep_t<5>(a, lds, p->stream);
        case 6: return launch_rsep_t<6>(a, lds, p->stream);
        case 7: return launch_rsep_t<7>(a, lds, p->stream);
        case 8: return launch_rsep_t<8>(a, lds, p->stream);
        case 9: return launch_rsep_t<9>(a, lds, p->stream);
        case 10: return launch_rsep_t<10>(a, lds, p->stream);
        case 11: return launch_rsep_t<11>(a, lds, p->stream);
        case 12: return launch_rsep_t<12>(a, lds, p->stream);
        case 13: return launch_rsep_t<13>(a, lds, p->stream);
        case 14: return launch_rsep_t<14>(a, lds, p->stream);
        default: return launch_rsep_t<15>(a, lds, p->stream);
    }
}

}  // namespace svc
