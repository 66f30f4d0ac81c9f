// Internal declarations of libsvconv: the plan object, launch descriptors and
// the host-side launchers of each kernel family.  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "svconv.h"

namespace svc {

constexpr int kMaxHalfWidth = 31;
constexpr int kMaxSpatialDegree = 6;
constexpr int kMaxSpatialTerms = (kMaxSpatialDegree + 1) * (kMaxSpatialDegree + 2) / 2;  // 28
constexpr int kMaxFilters = 64;      // filter rows one contraction launch handles
constexpr int kMaxCoefficients = 1024;

// Record a detail message for svconv_last_error and return the status.
int fail(int status, const std::string& msg);
// Map a HIP error to SVCONV_EDEVICE with a message (hipSuccess -> OK).
int hip_status(hipError_t e, const char* what);

// Dense filters in correlation orientation:
//   T_f(x,y) = sum_{dv,du} F[f][dv][du] X(x + du - h, y + dv - h).
// The basis form uses F_n[dv][du] = B_n[2h-dv][2h-du] (true convolution).

// Geometry of the tile the FP32 contraction works on.
struct F32Geometry {
    int k, n_rg, n_chunks;      // kernel width, 4-row groups, chunks = n_rg * k
    int nb;                     // 16-filter blocks
    int tile_w, tile_h;         // output tile
    int lds_rows, lds_cols, lds_pitch;
    size_t lds_bytes;
};

// Geometry of the low-precision (bf16/fp16) contraction.
struct LowpGeometry {
    int k, n_rg, n_q, n_steps;  // 4-row groups, 8-column chunks, steps = n_rg * n_q
    int nb;
    int tile_w, tile_h;
    int lds_rows, lds_pitch;    // pitch in 16-bit elements
    size_t lds_bytes;
};

// Arguments shared by the contraction kernels: input image X, per-pixel
// epilogue weights and the output.
struct ContractArgs {
    const float* X;             // [H][W]
    int H, W, h;
    int NF;                     // real filters (<= 16 * nb)
    int M, d_s;                 // spatial terms
    const float* coef;          // [NF][M] (basis form) or nullptr (weights are P_m)
    const double* beta;         // [NF] sum of each filter (pedestal restore), nullable
    const float* fscale;        // [NF] per-filter inverse scale, nullable
    float ped;
    double sx, ox, sy, oy;      // xh = sx * x + ox, yh = sy * y + oy (array x, y)
    const float* I;             // nullable
    float* out;                 // [H][W]; nullable when tout is set
    int y_begin = 0;            // output rows [y_begin, y_begin + n_rows)
    int n_rows = 0;
    float* tout = nullptr;      // optional T_f planes [NF][n_rows][W] (FP32 kernel only)
};

// Separable form (Gaussian bases only): one-dimensional factors per family.
constexpr int kSepMaxFactors = 10;   // degree <= 9 (N <= 64)
// spatial terms of the largest spatial degree (the padded coefficient stride)
constexpr int kSepCoefPad = (kMaxSpatialDegree + 1) * (kMaxSpatialDegree + 2) / 2;
struct SepArgs {
    const float* X;             // [H][W]
    const float* I;             // nullable
    float* out;                 // [H][W]
    int H, W, h;
    float ped;
    int G;                      // Gaussian families
    const int* fam;             // [2 G]: degree, index of the family's first basis
    const double* f1d;          // [G][kSepMaxFactors][k] factors f_e(w), w = -h..h
    const double* beta;         // [N] basis sums
    const float* coef;          // [N][M]
    const double* coefd;        // [N][M] float64 copy of coef (written by sep_prep)
    const double* gamma;        // [M] sum_n coef[n][m] beta[n] (written by sep_prep)
    const double* coefp;        // [N][kSepCoefPad] coefd padded with zeros beyond M (sep_prep)
    const double* gammap;       // [kSepCoefPad] gamma padded likewise (sep_prep)
    const float* coefpf;        // [N][kSepCoefPad] float32 copy of coefp (sep_prep)
    int M, d_s;
    int N;                      // bases (the adjoint in a)
    double sx, ox, sy, oy;
    int tiles_x, n_tiles;
    int y_begin, n_rows;        // output rows [y_begin, y_begin + n_rows)
    float* tout;                // nullable: T_n + s beta_n planes [N][n_rows][W] instead of D
    double* mom;                // adjoint in a on the matrix cores: [kSepMomCopies][N + 1][M] sums
};

// Regrouped separable form (separable_z.hip): the coefficients folded into
// per-call column filters g_{r,m} = sum_j a[n(r,j)][m] f_j, one row pass per
// row factor r and one column pass per (r, m) on the matrix cores.
constexpr int kSepZMaxHalfWidth = 12;
struct SepZArgs {
    const float* X;             // [H][W]
    const float* I;             // nullable
    float* out;                 // [H][W]
    int H, W, h;
    float ped;
    int R;                      // row factors of all families
    int M;                      // spatial terms (<= 6)
    double sx, ox, sy, oy;
    int tiles_x, n_tiles;
    int y_begin, n_rows;
    const int* rinfo;           // [2 R]: family, factor index
    const uint16_t* rtab;       // row-pass tap fragments of the precision
    const uint16_t* ztab;       // [R][3] per-call column-pass fragments
    const float* zinv;          // [6] 1 / (tap scale x data scale) per spatial term
    const double* gam;          // [kSepCoefPad] sum_n a[n][m] beta_n, zero-padded
};

// Regrouped contraction of small kernels on the vector units (direct.hip).
constexpr int kDirectMaxHalfWidth = 4;
struct DirectArgs {
    const float* X;             // [H][W]
    const float* I;             // nullable
    float* out;                 // [H][W]
    int H, W, h, d_s, M;
    float ped;
    const float* taps;          // Dirac delta basis: a [k^2][M]; otherwise Kt [M][k][k] (correlation order)
    double sx, ox, sy, oy;
    int tiles_x;
};

}  // namespace svc

struct svconv_plan {
    int H = 0, W = 0, h = 0, k = 0;
    int N = 0, d_s = 0, M = 0;
    int precision = SVCONV_FP32;
    int form = SVCONV_FORM_BASIS;
    bool dfb = false;                   // Dirac delta basis (one basis per kernel pixel)
    int bg = 0;                         // 1: the fit carries a background polynomial (M terms)
    int x0 = 0, y0 = 0, Wf = 0, Hf = 0;
    float pedestal = 0.f;
    hipStream_t stream = nullptr;
    int device = 0;

    std::vector<double> sigmas;
    std::vector<int> degrees;
    std::vector<double> basis;          // host B[n][v+h][u+h], float64
    double* dSep1d = nullptr;           // separable factors (Gaussian plans with h >= 1)
    int* dSepFam = nullptr;             // [2 G] degree, first basis
    double* dSepCoef = nullptr;         // [N + 1][kSepCoefPad] padded coefficients and gamma, then
                                        // the coefficients again in float32 (same layout)
    uint16_t* dSepFrag = nullptr;       // matrix-core Toeplitz fragments of the factors (fp16, bf16)
    double* dSepMom = nullptr;          // moment sums of the matrix-core adjoint in a
    int sepR = 0;                       // row factors of all families
    int* dSepRinfo = nullptr;           // [2 sepR] family, factor index of each row factor
    uint16_t* dSepZRow = nullptr;       // regrouped separable form: row-pass fragments (fp16, bf16)
    uint16_t* dSepZTab = nullptr;       // per-call column-pass fragments
    float* dSepZInv = nullptr;          // [8] per-call inverse scales
    double* dSepZGam = nullptr;         // [kSepCoefPad] per-call pedestal sums

    // device tables (basis form, fixed per plan)
    float* dF32 = nullptr;              // [N][k][k] correlation-oriented basis, float32
    double* dF64 = nullptr;             // same, float64
    double* dBeta = nullptr;            // [N] sums
    float* dFragF32 = nullptr;          // FP32 MFMA A-operand fragments
    uint16_t* dFragLoB = nullptr;       // bf16 fragments, hi then lo halves
    uint16_t* dFragLoH = nullptr;       // fp16 fragments, hi then lo halves
    float* dScaleB = nullptr;           // [2][kMaxFilters] scales / inverse scales, bf16 fragments
    float* dScaleH = nullptr;           // [2][kMaxFilters] scales / inverse scales, fp16 fragments

    // per-call scratch (allocated once)
    float* dFt32 = nullptr;             // [kMaxFilters][k][k] per-call filters (regrouped / adjoint)
    double* dBetaT = nullptr;           // [kMaxFilters]
    float* dFragT32 = nullptr;          // fragments of per-call filters (FP32)
    uint16_t* dFragTB = nullptr;        // per-call bf16 fragments
    uint16_t* dFragTH = nullptr;        // per-call fp16 fragments
    float* dScaleT = nullptr;           // [2][kMaxFilters] per-call scales / inverse scales
    double* dQpart = nullptr;           // adjoint-a partials
    int q_blocks = 0;                   // number of partial blocks
    double* dQ = nullptr;               // reduced Q [M][k*k]
    float* dGrad = nullptr;             // [H][W] float scratch (loss gradient)
    double* dVec = nullptr;             // small float64 scratch (fit)
    int* dStatus = nullptr;             // device status word
    double* dNMpart = nullptr;          // normal-matrix partials and totals
    float* dTband = nullptr;            // basis responses of a band of rows (normal matrix)
    size_t tband_bytes = 0, nmpart_bytes = 0;
    double* dRed = nullptr;             // reduction scratch (loss)
};

namespace svc {

// forward.hip
size_t f32_fragment_floats(int k, int nb);
size_t lowp_fragment_elems(int k, int nb);  // hi and lo halves together
F32Geometry f32_geometry(int k, int nb);
LowpGeometry lowp_geometry(int k, int nb);
// With at most 8 filters (f32_packed) the FP32 fragments and contraction take
// the two-row packed layout; both sides decide it from NF alone, so a fragment
// buffer built for NF filters serves every launch with the same NF.
bool f32_packed(int NF);
int build_f32_fragments(const float* F, int NF, int k, float* frag, hipStream_t s);
int build_lowp_fragments(const float* F, int NF, int k, int fp16, float* scale,
                         uint16_t* frag, hipStream_t s, bool packed = false);
// true when launch_contract_lowp runs the two-column packed kernel for these
// arguments (regrouped filters, at most 8 of them); its fragments must then be
// built with packed = true
bool lowp_packed(const ContractArgs& a, int nb);
int regroup_filters(const double* F64, const double* beta, const float* a, int N, int M, int k,
                    float* Ft, double* betaT, hipStream_t s);
int adjoint_filters(const double* F64, const float* a, int N, int M, int d_s, int k,
                    double sx, double sy, float* Ft, hipStream_t s);
int launch_contract_f32(const ContractArgs& a, const float* frag, int nb, hipStream_t s);
int launch_contract_lowp(const ContractArgs& a, const uint16_t* frag, int nb, int precision,
                         hipStream_t s);

// separable.hip, separable_adjoint.hip
int launch_contract_sep(SepArgs a, hipStream_t s);
int launch_sep_prep(const float* coef, const double* beta, int N, int M, double* coefd,
                    double* gamma, double* coefp, hipStream_t s);
size_t sep_mma_frag_entries(int G);
int build_sep_mma_fragments(const double* f1d, int G, int h, uint16_t* frag, hipStream_t s);
int launch_contract_sep_mma(SepArgs a, const uint16_t* frag, int precision, hipStream_t s);
// adjoint in R through the separable factors on the matrix cores (bf16x3); a.X = G, a.out = dL/dR
int launch_adjoint_r_sep_mma(SepArgs a, const uint16_t* frag, hipStream_t s);
// adjoint in a through the separable factors on the matrix cores: a.X = R, a.I = G,
// ga[n][m] = sum_p G P_m T_n (the split precision's products) + s beta_n sum_p G P_m
constexpr int kSepMomCopies = 8;        // copies of the moment sums the tiles spread their atomics over
int launch_adjoint_a_sep_mma(SepArgs a, const uint16_t* frag, int precision, const double* beta,
                             double* ga, hipStream_t s);
int launch_adjoint_a_sep(svconv_plan* p, const float* R, const float* G, double* ga);
bool sep_adjoint_supported(const svconv_plan* p);
int launch_adjoint_r_sep(svconv_plan* p, const float* a32, const float* G, float* gR);

// separable_z.hip
size_t sepz_rtab_entries(int R);    // both precisions
size_t sepz_ztab_entries(int R);
// only: -1 builds both precisions (fp16 then bf16), 0 only fp16, 1 only bf16
int build_sepz_rtab(const double* f1d, const int* rinfo, int R, int h, uint16_t* rtab, hipStream_t s,
                    int only = -1);
int launch_sepz_prep(const SepZArgs& z, const float* a, const double* f1d, const int* fam, const double* beta, int N,
                     bool fp16, hipStream_t s);
int launch_contract_sepz(SepZArgs a, int precision, hipStream_t s);

// direct.hip
bool direct_supported(int h, int d_s);
int launch_contract_direct(DirectArgs a, bool dfb, hipStream_t s);

// Both separable forms go through the one-dimensional factors in the adjoints
// and the fit.
inline bool sep_form(const svconv_plan* p) {
    return p->form == SVCONV_FORM_SEPARABLE || p->form == SVCONV_FORM_SEPARABLE_REGROUPED;
}

// plan.hip
int run_forward(svconv_plan* p, const float* R, const float* I, const float* a, float* out);

// backward.hip
size_t adjoint_scratch_doubles(int H, int W, int k, int M);
int launch_adjoint_a(svconv_plan* p, const float* R, const float* gD, double* ga);

// fit.hip
int launch_loss_grad(svconv_plan* p, const float* D, const unsigned char* mask, float* gD,
                     double* loss);
int launch_normal_matrix(svconv_plan* p, const float* R, const float* I, const unsigned char* mask,
                         double* JtJ, double* rhs);
int launch_ls_grad(svconv_plan* p, const double* A, const double* a64, const double* rhs, double* g, int n);
int launch_cholesky(svconv_plan* p, double* A, int n);
int launch_cholesky_solve(svconv_plan* p, const double* L, const double* rhs, double* x, int n);
int launch_gn_update(svconv_plan* p, const double* delta, double* a64, float* a32, int n);
int launch_copy_a(svconv_plan* p, const double* a64, float* a32, int n);
int launch_scale(svconv_plan* p, double* v, double s, int n);

// ois.hip
int launch_add_background(svconv_plan* p, const float* b, float* D);
int launch_bg_grad(svconv_plan* p, const float* G, double* gb);

}  // namespace svc
