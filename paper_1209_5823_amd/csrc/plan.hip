// C ABI of libsvconv: plan construction (float64 basis on the host,
// device tables), argument validation and dispatch to the kernel families.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>

#include "internal.hpp"

namespace svc {

static thread_local std::string g_last_error;

int fail(int status, const std::string& msg) {
    g_last_error = msg;
    return status;
}

int hip_status(hipError_t e, const char* what) {
    if (e == hipSuccess) return SVCONV_OK;
    return fail(SVCONV_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// Basis functions (Sec. 2, Eq. 2; Gaussian basis of Alard & Lupton):
// Gaussian of width sigma times u^i v^j, unit L1 norm; sigma = 0 is a delta.
// Layout B[n][v+h][u+h].
static void build_basis(int h, const std::vector<double>& sig, const std::vector<int>& deg,
                        std::vector<double>& B) {
    const int k = 2 * h + 1;
    B.clear();
    for (size_t g = 0; g < sig.size(); ++g) {
        for (int t = 0; t <= deg[g]; ++t) {
            for (int i = t; i >= 0; --i) {
                const int j = t - i;
                std::vector<double> b((size_t)k * k);
                double l1 = 0.0;
                for (int v = -h; v <= h; ++v) {
                    for (int u = -h; u <= h; ++u) {
                        double val;
                        if (sig[g] == 0.0) {
                            val = (u == 0 && v == 0) ? 1.0 : 0.0;
                        } else {
                            double mono = 1.0;
                            for (int q = 0; q < i; ++q) mono *= u;
                            for (int q = 0; q < j; ++q) mono *= v;
                            val = std::exp(-(double)(u * u + v * v) / (2.0 * sig[g] * sig[g])) * mono;
                        }
                        b[(size_t)(v + h) * k + (u + h)] = val;
                        l1 += std::fabs(val);
                    }
                }
                if (l1 > 0.0)
                    for (auto& q : b) q /= l1;
                B.insert(B.end(), b.begin(), b.end());
            }
        }
    }
}

template <class T>
static int dalloc(T** p, size_t count, const char* what) {
    *p = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMalloc((void**)p, count * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(SVCONV_ENOMEM, std::string("hipMalloc failed for ") + what);
    }
    return SVCONV_OK;
}

static void free_plan(svconv_plan* p) {
    void* ptrs[] = {p->dSep1d, p->dSepFam, p->dSepCoef, p->dSepFrag, p->dSepMom, p->dSepRinfo,
                    p->dSepZRow, p->dSepZTab, p->dSepZInv, p->dSepZGam,
                    p->dF32,   p->dF64,   p->dBeta,   p->dFragF32, p->dFragLoB, p->dFragLoH,
                    p->dScaleB, p->dScaleH, p->dFt32, p->dBetaT, p->dFragT32, p->dFragTB,  p->dFragTH,
                    p->dScaleT, p->dQpart, p->dQ,    p->dGrad,    p->dVec,     p->dStatus,
                    p->dNMpart, p->dTband, p->dRed};
    for (void* q : ptrs)
        if (q) (void)hipFree(q);
    delete p;
}

static void coords(const svconv_plan* p, ContractArgs& a) {
    // xh = 2 (x + x0) / (Wf - 1) - 1 = sx * x + ox; 0 on a one-pixel axis
    if (p->Wf > 1) {
        a.sx = 2.0 / (p->Wf - 1);
        a.ox = a.sx * p->x0 - 1.0;
    } else {
        a.sx = 0.0;
        a.ox = 0.0;
    }
    if (p->Hf > 1) {
        a.sy = 2.0 / (p->Hf - 1);
        a.oy = a.sy * p->y0 - 1.0;
    } else {
        a.sy = 0.0;
        a.oy = 0.0;
    }
}

static bool is_lowp(int precision) { return precision >= SVCONV_BF16 && precision <= SVCONV_FP16X3; }
static bool is_fp16(int precision) {
    return precision == SVCONV_FP16 || precision == SVCONV_FP16X2 || precision == SVCONV_FP16X3;
}

}  // namespace svc

using namespace svc;

// Device tables, scratch and basis-form fragments of a plan whose sizes and
// host basis table are set.
static int finish_plan(svconv_plan* p, svconv_plan** out) {
    p->Wf = p->W;
    p->Hf = p->H;

    int st = hip_status(hipGetDevice(&p->device), "hipGetDevice");
    if (st) { free_plan(p); return st; }

    const int k = p->k, kk = k * k;
    // correlation-oriented tables: F_n[dv][du] = B_n[2h-dv][2h-du]
    std::vector<float> F32((size_t)p->N * kk);
    std::vector<double> F64((size_t)p->N * kk), beta(p->N);
    for (int n = 0; n < p->N; ++n) {
        double s = 0.0;
        for (int dv = 0; dv < k; ++dv)
            for (int du = 0; du < k; ++du) {
                const double b = p->basis[(size_t)n * kk + (size_t)(k - 1 - dv) * k + (k - 1 - du)];
                F64[(size_t)n * kk + dv * k + du] = b;
                F32[(size_t)n * kk + dv * k + du] = (float)b;
                s += b;
            }
        beta[n] = s;
    }

    // basis-form fragment tables exist only for N <= 64 (a delta basis with
    // more kernel pixels is contracted in the regrouped form only)
    const int nbN = p->N <= kMaxFilters ? (p->N + 15) / 16 : 1;
    const size_t frag32 = f32_fragment_floats(k, nbN);
    const size_t fragT32 = f32_fragment_floats(k, (kMaxSpatialTerms + 15) / 16);
    const size_t fraglN = lowp_fragment_elems(k, nbN);
    const size_t fraglT = lowp_fragment_elems(k, (kMaxSpatialTerms + 15) / 16);
    if ((st = dalloc(&p->dF32, F32.size(), "basis table")) ||
        (st = dalloc(&p->dF64, F64.size(), "basis table (f64)")) ||
        (st = dalloc(&p->dBeta, beta.size(), "basis sums")) ||
        (st = dalloc(&p->dFragF32, frag32, "fp32 fragments")) ||
        (st = dalloc(&p->dFragLoB, fraglN, "bf16 fragments")) ||
        (st = dalloc(&p->dFragLoH, fraglN, "fp16 fragments")) ||
        (st = dalloc(&p->dScaleB, (size_t)2 * kMaxFilters, "bf16 scales")) ||
        (st = dalloc(&p->dScaleH, (size_t)2 * kMaxFilters, "fp16 scales")) ||
        (st = dalloc(&p->dFt32, (size_t)kMaxFilters * kk, "per-call filters")) ||
        (st = dalloc(&p->dBetaT, (size_t)kMaxFilters, "per-call sums")) ||
        (st = dalloc(&p->dFragT32, fragT32, "per-call fp32 fragments")) ||
        (st = dalloc(&p->dFragTB, fraglT, "per-call bf16 fragments")) ||
        (st = dalloc(&p->dFragTH, fraglT, "per-call fp16 fragments")) ||
        (st = dalloc(&p->dScaleT, (size_t)2 * kMaxFilters, "per-call scales")) ||
        (st = dalloc(&p->dVec, (size_t)8 * kMaxCoefficients + 64, "vector scratch")) ||
        (st = dalloc(&p->dStatus, (size_t)4, "status word")) ||
        (st = dalloc(&p->dGrad, (size_t)p->H * p->W, "loss gradient")) ||
        (st = dalloc(&p->dRed, (size_t)2048, "reduction scratch")) ||
        (st = dalloc(&p->dQpart, adjoint_scratch_doubles(p->H, p->W, p->k, p->M), "adjoint scratch"))) {
        free_plan(p);
        return st;
    }
    st = hip_status(hipMemcpy(p->dF32, F32.data(), F32.size() * 4, hipMemcpyHostToDevice), "upload");
    if (!st) st = hip_status(hipMemcpy(p->dF64, F64.data(), F64.size() * 8, hipMemcpyHostToDevice), "upload");
    if (!st) st = hip_status(hipMemcpy(p->dBeta, beta.data(), beta.size() * 8, hipMemcpyHostToDevice), "upload");
    if (!st && !p->dfb && p->h >= 1) {
        // one-dimensional factors of every Gaussian family (the separable form)
        const int G = (int)p->sigmas.size(), h = p->h;
        std::vector<double> f1d((size_t)G * kSepMaxFactors * k, 0.0);
        std::vector<int> fam(2 * (size_t)G);
        int first = 0;
        for (int g = 0; g < G; ++g) {
            fam[2 * g] = p->degrees[g];
            fam[2 * g + 1] = first;
            first += (p->degrees[g] + 1) * (p->degrees[g] + 2) / 2;
            for (int e = 0; e <= p->degrees[g]; ++e) {
                double* f = &f1d[((size_t)g * kSepMaxFactors + e) * k];
                double l1 = 0.0;
                for (int w = -h; w <= h; ++w) {
                    double val;
                    if (p->sigmas[g] == 0.0) {
                        val = (w == 0) ? 1.0 : 0.0;
                    } else {
                        double mono = 1.0;
                        for (int q = 0; q < e; ++q) mono *= w;
                        val = std::exp(-(double)(w * w) / (2.0 * p->sigmas[g] * p->sigmas[g])) * mono;
                    }
                    f[w + h] = val;
                    l1 += std::fabs(val);
                }
                if (l1 > 0.0)
                    for (int q = 0; q < k; ++q) f[q] /= l1;
            }
        }
        st = dalloc(&p->dSep1d, f1d.size(), "separable factors");
        if (!st) st = dalloc(&p->dSepFam, fam.size(), "separable families");
        // float64 table then its float32 copy (the matrix-core epilogue)
        if (!st) st = dalloc(&p->dSepCoef, 2 * (size_t)(p->N + 1) * kSepCoefPad, "separable coefficients");
        if (!st) st = hip_status(hipMemcpy(p->dSep1d, f1d.data(), f1d.size() * 8, hipMemcpyHostToDevice), "upload");
        if (!st) st = hip_status(hipMemcpy(p->dSepFam, fam.data(), fam.size() * 4, hipMemcpyHostToDevice), "upload");
        if (!st && h <= 15) {
            st = dalloc(&p->dSepFrag, sep_mma_frag_entries(G), "separable matrix-core fragments");
            if (!st) st = build_sep_mma_fragments(p->dSep1d, G, h, p->dSepFrag, nullptr);
            if (!st) st = dalloc(&p->dSepMom, (size_t)kSepMomCopies * (p->N + 1) * p->M, "separable moments");
        }
        if (!st && h <= kSepZMaxHalfWidth && p->d_s <= 2) {
            // the regrouped separable form: row factors of all families in order
            std::vector<int> rinfo;
            for (int g = 0; g < G; ++g)
                for (int i = 0; i <= p->degrees[g]; ++i) {
                    rinfo.push_back(g);
                    rinfo.push_back(i);
                }
            p->sepR = (int)(rinfo.size() / 2);
            st = dalloc(&p->dSepRinfo, rinfo.size(), "row factors");
            if (!st) st = hip_status(hipMemcpy(p->dSepRinfo, rinfo.data(), rinfo.size() * 4, hipMemcpyHostToDevice),
                                     "upload");
            if (!st) st = dalloc(&p->dSepZRow, sepz_rtab_entries(p->sepR), "row-pass fragments");
            if (!st) st = dalloc(&p->dSepZTab, sepz_ztab_entries(p->sepR), "column-pass fragments");
            if (!st) st = dalloc(&p->dSepZInv, (size_t)8, "column-pass scales");
            if (!st) st = dalloc(&p->dSepZGam, (size_t)kSepCoefPad, "pedestal sums");
            if (!st) st = build_sepz_rtab(p->dSep1d, p->dSepRinfo, p->sepR, h, p->dSepZRow, nullptr);
        }
    }
    if (!st && p->N <= kMaxFilters) {
        st = build_f32_fragments(p->dF32, p->N, k, p->dFragF32, nullptr);
        if (!st) st = build_lowp_fragments(p->dF32, p->N, k, 0, p->dScaleB, p->dFragLoB, nullptr);
        if (!st) st = build_lowp_fragments(p->dF32, p->N, k, 1, p->dScaleH, p->dFragLoH, nullptr);
    }
    if (!st) st = hip_status(hipDeviceSynchronize(), "plan table build");
    if (st) { free_plan(p); return st; }
    *out = p;
    return SVCONV_OK;
}

namespace svc {

// Shared body of svconv_forward, svconv_difference, svconv_gn_step and the
// tile pipeline: enqueue one forward pass on the plan's stream.
int run_forward(svconv_plan* p, const float* R, const float* I, const float* a, float* out) {
    ContractArgs c{};
    c.X = R;
    c.H = p->H;
    c.W = p->W;
    c.h = p->h;
    c.M = p->M;
    c.d_s = p->d_s;
    c.ped = p->pedestal;
    c.I = I;
    c.out = out;
    c.y_begin = 0;
    c.n_rows = p->H;
    coords(p, c);
    const bool lowp = is_lowp(p->precision);
    if (p->form == SVCONV_FORM_SEPARABLE_REGROUPED) {
        const bool split = p->precision == SVCONV_FP16X3 || p->precision == SVCONV_BF16X3 ||
                           p->precision == SVCONV_FP16X2;
        if (!split) return fail(SVCONV_EUNSUPPORTED, "regrouped separable form needs a split 16-bit precision");
        if (!p->dSepZRow) return fail(SVCONV_EUNSUPPORTED, "regrouped separable form needs 1 <= half-width <= 12 "
                                                          "and spatial degree <= 2");
        SepZArgs z{};
        z.X = R;
        z.I = I;
        z.out = out;
        z.H = p->H;
        z.W = p->W;
        z.h = p->h;
        z.ped = p->pedestal;
        z.R = p->sepR;
        z.M = p->M;
        z.sx = c.sx; z.ox = c.ox; z.sy = c.sy; z.oy = c.oy;
        z.y_begin = 0;
        z.n_rows = p->H;
        z.rinfo = p->dSepRinfo;
        const bool h16 = is_fp16(p->precision);
        z.rtab = p->dSepZRow + (h16 ? 0 : sepz_rtab_entries(p->sepR) / 2);
        z.ztab = p->dSepZTab;
        z.zinv = p->dSepZInv;
        z.gam = p->dSepZGam;
        int st = launch_sepz_prep(z, a, p->dSep1d, p->dSepFam, p->dBeta, p->N, h16, p->stream);
        if (st) return st;
        return launch_contract_sepz(z, p->precision, p->stream);
    }
    if (p->form == SVCONV_FORM_SEPARABLE) {
        SepArgs sa{};
        sa.X = R;
        sa.I = I;
        sa.out = out;
        sa.H = p->H;
        sa.W = p->W;
        sa.h = p->h;
        sa.ped = p->pedestal;
        sa.G = (int)p->sigmas.size();
        sa.fam = p->dSepFam;
        sa.f1d = p->dSep1d;
        sa.beta = p->dBeta;
        sa.coef = a;
        sa.M = p->M;
        sa.d_s = p->d_s;
        sa.sx = c.sx; sa.ox = c.ox; sa.sy = c.sy; sa.oy = c.oy;
        sa.y_begin = 0;
        sa.n_rows = p->H;
        sa.tout = nullptr;
        // per-call tables in the plan's vector scratch, past what the fit uses
        double* coefd = p->dVec + 7 * (size_t)kMaxCoefficients;
        double* gamma = p->dVec + 8 * (size_t)kMaxCoefficients;
        int st = launch_sep_prep(a, p->dBeta, p->N, p->M, coefd, gamma, p->dSepCoef, p->stream);
        if (st) return st;
        sa.coefd = coefd;
        sa.gamma = gamma;
        sa.coefp = p->dSepCoef;
        sa.gammap = p->dSepCoef + (size_t)p->N * kSepCoefPad;
        sa.coefpf = reinterpret_cast<const float*>(p->dSepCoef + (size_t)(p->N + 1) * kSepCoefPad);
        // the split 16-bit precisions take the matrix-core passes, the others float64
        if (p->precision == SVCONV_FP16X3 || p->precision == SVCONV_BF16X3 || p->precision == SVCONV_FP16X2) {
            if (!p->dSepFrag) return fail(SVCONV_EUNSUPPORTED, "separable matrix-core form needs half-width <= 15");
            return launch_contract_sep_mma(sa, p->dSepFrag, p->precision, p->stream);
        }
        return launch_contract_sep(sa, p->stream);
    }
    if (p->form == SVCONV_FORM_BASIS) {
        if (p->N > kMaxFilters) return fail(SVCONV_EUNSUPPORTED, "basis form needs N <= 64");
        c.NF = p->N;
        c.coef = a;
        c.beta = p->dBeta;
        const int nb = (p->N + 15) / 16;
        if (!lowp) return launch_contract_f32(c, p->dFragF32, nb, p->stream);
        c.fscale = (is_fp16(p->precision) ? p->dScaleH : p->dScaleB) + kMaxFilters;
        return launch_contract_lowp(c, is_fp16(p->precision) ? p->dFragLoH : p->dFragLoB, nb,
                                    p->precision, p->stream);
    }
    // regrouped: Kt_m built on the device for this call (the delta basis' Kt_m
    // is a itself); small kernels in float32 on the vector units
    if (!lowp && direct_supported(p->h, p->d_s)) {
        DirectArgs d{};
        d.X = R;
        d.I = I;
        d.out = out;
        d.H = p->H;
        d.W = p->W;
        d.h = p->h;
        d.d_s = p->d_s;
        d.M = p->M;
        d.ped = p->pedestal;
        d.sx = c.sx; d.ox = c.ox; d.sy = c.sy; d.oy = c.oy;
        if (p->dfb) {
            d.taps = a;
            return launch_contract_direct(d, true, p->stream);
        }
        int st = regroup_filters(p->dF64, p->dBeta, a, p->N, p->M, p->k, p->dFt32, p->dBetaT, p->stream);
        if (st) return st;
        d.taps = p->dFt32;
        return launch_contract_direct(d, false, p->stream);
    }
    if (p->M > 32) return fail(SVCONV_EUNSUPPORTED, "regrouped form needs M <= 32");
    int st = regroup_filters(p->dF64, p->dBeta, a, p->N, p->M, p->k, p->dFt32, p->dBetaT, p->stream);
    if (st) return st;
    c.NF = p->M;
    c.coef = nullptr;
    c.beta = p->dBetaT;
    const int nb = (p->M + 15) / 16;
    if (!lowp) {
        st = build_f32_fragments(p->dFt32, p->M, p->k, p->dFragT32, p->stream);
        if (st) return st;
        return launch_contract_f32(c, p->dFragT32, nb, p->stream);
    }
    const bool h16 = is_fp16(p->precision);
    uint16_t* frag = h16 ? p->dFragTH : p->dFragTB;
    c.fscale = p->dScaleT + kMaxFilters;
    st = build_lowp_fragments(p->dFt32, p->M, p->k, h16 ? 1 : 0, p->dScaleT, frag, p->stream,
                              lowp_packed(c, nb));
    if (st) return st;
    return launch_contract_lowp(c, frag, nb, p->precision, p->stream);
}

}  // namespace svc

extern "C" {

const char* svconv_strerror(int status) {
    switch (status) {
        case SVCONV_OK: return "success";
        case SVCONV_EINVAL: return "invalid argument";
        case SVCONV_ENOMEM: return "out of memory";
        case SVCONV_EDEVICE: return "device (HIP) error";
        case SVCONV_EUNSUPPORTED: return "unsupported configuration";
        case SVCONV_ENOTSPD: return "matrix is not symmetric positive definite";
        default: return "unknown status";
    }
}

const char* svconv_last_error(void) { return g_last_error.c_str(); }

int svconv_plan_create(svconv_plan** out, int height, int width, int half_width, int n_gauss,
                       const double* sigmas, const int* degrees, int spatial_degree,
                       int precision) {
    g_last_error.clear();
    if (!out) return fail(SVCONV_EINVAL, "out is NULL");
    *out = nullptr;
    if (height <= 0 || width <= 0) return fail(SVCONV_EINVAL, "image size must be positive");
    if (half_width < 0) return fail(SVCONV_EINVAL, "half_width < 0");
    if (n_gauss <= 0 || !sigmas || !degrees) return fail(SVCONV_EINVAL, "no basis families");
    if (spatial_degree < 0) return fail(SVCONV_EINVAL, "spatial_degree < 0");
    if (precision < SVCONV_FP32 || precision > SVCONV_FP16X3)
        return fail(SVCONV_EINVAL, "unknown precision");
    long N = 0;
    for (int g = 0; g < n_gauss; ++g) {
        if (!(sigmas[g] >= 0.0) || !std::isfinite(sigmas[g]))
            return fail(SVCONV_EINVAL, "sigma must be finite and >= 0");
        if (degrees[g] < 0) return fail(SVCONV_EINVAL, "degree < 0");
        if (sigmas[g] == 0.0 && degrees[g] != 0)
            return fail(SVCONV_EINVAL, "a delta basis (sigma 0) must have degree 0");
        if (degrees[g] > 64) return fail(SVCONV_EINVAL, "degree too large");
        N += (long)(degrees[g] + 1) * (degrees[g] + 2) / 2;
    }
    if (half_width > kMaxHalfWidth) return fail(SVCONV_EUNSUPPORTED, "half_width > 31");
    if (spatial_degree > kMaxSpatialDegree) return fail(SVCONV_EUNSUPPORTED, "spatial_degree > 6");
    const int M = (spatial_degree + 1) * (spatial_degree + 2) / 2;
    if (N * M > kMaxCoefficients) return fail(SVCONV_EUNSUPPORTED, "N * M > 1024");
    if (N > kMaxFilters) return fail(SVCONV_EUNSUPPORTED, "more than 64 basis functions");

    svconv_plan* p = new (std::nothrow) svconv_plan();
    if (!p) return fail(SVCONV_ENOMEM, "host allocation of the plan");
    p->H = height;
    p->W = width;
    p->h = half_width;
    p->k = 2 * half_width + 1;
    p->N = (int)N;
    p->d_s = spatial_degree;
    p->M = M;
    p->precision = precision;
    p->sigmas.assign(sigmas, sigmas + n_gauss);
    p->degrees.assign(degrees, degrees + n_gauss);
    build_basis(p->h, p->sigmas, p->degrees, p->basis);
    return finish_plan(p, out);
}

// Dirac delta basis (Sec. 2: one basis function per kernel pixel): basis n =
// (v + h) k + (u + h) is 1 at (u, v) and 0 elsewhere, so K(x,y)[u,v] =
// sum_m a[n(u,v)][m] P_m(x,y).
int svconv_plan_create_dfb(svconv_plan** out, int height, int width, int half_width,
                           int spatial_degree, int precision) {
    g_last_error.clear();
    if (!out) return fail(SVCONV_EINVAL, "out is NULL");
    *out = nullptr;
    if (height <= 0 || width <= 0) return fail(SVCONV_EINVAL, "image size must be positive");
    if (half_width < 0) return fail(SVCONV_EINVAL, "half_width < 0");
    if (spatial_degree < 0) return fail(SVCONV_EINVAL, "spatial_degree < 0");
    if (precision < SVCONV_FP32 || precision > SVCONV_FP16X3)
        return fail(SVCONV_EINVAL, "unknown precision");
    if (half_width > kMaxHalfWidth) return fail(SVCONV_EUNSUPPORTED, "half_width > 31");
    if (spatial_degree > kMaxSpatialDegree) return fail(SVCONV_EUNSUPPORTED, "spatial_degree > 6");
    const int M = (spatial_degree + 1) * (spatial_degree + 2) / 2;
    const long k = 2L * half_width + 1;
    const long N = k * k;
    if (N * M > kMaxCoefficients) return fail(SVCONV_EUNSUPPORTED, "N * M > 1024");
    svconv_plan* p = new (std::nothrow) svconv_plan();
    if (!p) return fail(SVCONV_ENOMEM, "host allocation of the plan");
    p->H = height;
    p->W = width;
    p->h = half_width;
    p->k = (int)k;
    p->N = (int)N;
    p->d_s = spatial_degree;
    p->M = M;
    p->precision = precision;
    p->dfb = true;
    p->form = SVCONV_FORM_REGROUPED;
    p->basis.assign((size_t)N * N, 0.0);
    for (long n = 0; n < N; ++n) p->basis[(size_t)n * N + n] = 1.0;
    return finish_plan(p, out);
}

int svconv_plan_set_frame(svconv_plan* p, int x0, int y0, int frame_width, int frame_height) {
    if (!p) return fail(SVCONV_EINVAL, "plan is NULL");
    if (x0 < 0 || y0 < 0 || frame_width <= 0 || frame_height <= 0 ||
        (long)x0 + p->W > frame_width || (long)y0 + p->H > frame_height)
        return fail(SVCONV_EINVAL, "image does not lie inside the frame");
    p->x0 = x0;
    p->y0 = y0;
    p->Wf = frame_width;
    p->Hf = frame_height;
    return SVCONV_OK;
}

int svconv_plan_set_stream(svconv_plan* p, void* stream) {
    if (!p) return fail(SVCONV_EINVAL, "plan is NULL");
    p->stream = (hipStream_t)stream;
    return SVCONV_OK;
}

int svconv_plan_set_precision(svconv_plan* p, int precision) {
    if (!p) return fail(SVCONV_EINVAL, "plan is NULL");
    if (precision < SVCONV_FP32 || precision > SVCONV_FP16X3)
        return fail(SVCONV_EINVAL, "unknown precision");
    p->precision = precision;
    return SVCONV_OK;
}

int svconv_plan_set_form(svconv_plan* p, int form) {
    if (!p) return fail(SVCONV_EINVAL, "plan is NULL");
    if (form != SVCONV_FORM_BASIS && form != SVCONV_FORM_REGROUPED && form != SVCONV_FORM_SEPARABLE &&
        form != SVCONV_FORM_SEPARABLE_REGROUPED)
        return fail(SVCONV_EINVAL, "unknown form");
    if (form == SVCONV_FORM_SEPARABLE_REGROUPED && !p->dSepZRow)
        return fail(SVCONV_EUNSUPPORTED, "regrouped separable form needs Gaussian bases, 1 <= half-width <= 12 "
                                         "and spatial degree <= 2");
    if (form == SVCONV_FORM_SEPARABLE && (!p->dSep1d || p->h > 15))
        return fail(SVCONV_EUNSUPPORTED, "separable form needs Gaussian bases and 1 <= half-width <= 15");
    if (form == SVCONV_FORM_BASIS && p->N > kMaxFilters)
        return fail(SVCONV_EUNSUPPORTED, "basis form needs N <= 64");
    p->form = form;
    return SVCONV_OK;
}

int svconv_plan_set_pedestal(svconv_plan* p, float pedestal) {
    if (!p) return fail(SVCONV_EINVAL, "plan is NULL");
    if (!std::isfinite(pedestal)) return fail(SVCONV_EINVAL, "pedestal must be finite");
    p->pedestal = pedestal;
    return SVCONV_OK;
}

int svconv_plan_sizes(const svconv_plan* p, int* n_basis, int* n_spatial) {
    if (!p) return fail(SVCONV_EINVAL, "plan is NULL");
    if (n_basis) *n_basis = p->N;
    if (n_spatial) *n_spatial = p->M;
    return SVCONV_OK;
}

int svconv_plan_get_basis(const svconv_plan* p, double* host_out) {
    if (!p || !host_out) return fail(SVCONV_EINVAL, "NULL argument");
    std::memcpy(host_out, p->basis.data(), p->basis.size() * sizeof(double));
    return SVCONV_OK;
}

int svconv_plan_destroy(svconv_plan* p) {
    if (!p) return SVCONV_OK;
    int st = hip_status(hipStreamSynchronize(p->stream), "hipStreamSynchronize");
    free_plan(p);
    return st;
}

int svconv_forward(svconv_plan* p, const float* R, const float* a, float* out) {
    if (!p || !R || !a || !out) return fail(SVCONV_EINVAL, "NULL argument");
    if ((const void*)out == (const void*)R) return fail(SVCONV_EINVAL, "out aliases R");
    return run_forward(p, R, nullptr, a, out);
}

int svconv_difference(svconv_plan* p, const float* R, const float* I, const float* a, float* D) {
    if (!p || !R || !I || !a || !D) return fail(SVCONV_EINVAL, "NULL argument");
    if ((const void*)D == (const void*)R) return fail(SVCONV_EINVAL, "D aliases R");
    return run_forward(p, R, I, a, D);
}

// Adjoint in a: with the separable form at a split precision, the forward's
// matrix-core passes with moment sums in place of the epilogue; otherwise the
// float64 separable kernel or the dense product.
static int run_adjoint_a(svconv_plan* p, const float* R, const float* gD, double* ga) {
    if (sep_form(p) && (p->precision == SVCONV_FP16X3 || p->precision == SVCONV_BF16X3) &&
        p->dSepFrag && p->dSepMom) {
        ContractArgs c{};
        coords(p, c);
        SepArgs sa{};
        sa.X = R;
        sa.I = gD;
        sa.H = p->H;
        sa.W = p->W;
        sa.h = p->h;
        sa.ped = p->pedestal;
        sa.G = (int)p->sigmas.size();
        sa.fam = p->dSepFam;
        sa.M = p->M;
        sa.d_s = p->d_s;
        sa.sx = c.sx; sa.ox = c.ox; sa.sy = c.sy; sa.oy = c.oy;
        sa.y_begin = 0;
        sa.n_rows = p->H;
        sa.N = p->N;
        sa.mom = p->dSepMom;
        return launch_adjoint_a_sep_mma(sa, p->dSepFrag, p->precision, p->dBeta, ga, p->stream);
    }
    return launch_adjoint_a(p, R, gD, ga);
}

int svconv_backward(svconv_plan* p, const float* R, const float* a, const float* gD, float* gR,
                    double* ga) {
    if (!p || !R || !a || !gD) return fail(SVCONV_EINVAL, "NULL argument");
    if (gR && ((const void*)gR == (const void*)R || (const void*)gR == (const void*)gD))
        return fail(SVCONV_EINVAL, "gR aliases R or gD");
    if (p->M > 32) return fail(SVCONV_EUNSUPPORTED, "adjoint in R needs M <= 32");
    int st = SVCONV_OK;
    if (gR && sep_form(p) &&
        (p->precision == SVCONV_FP16X3 || p->precision == SVCONV_BF16X3) && p->dSepFrag) {
        // through the separable factors on the matrix cores (bf16x3 for both split
        // precisions: bf16 keeps the float32 range of c_n gD)
        ContractArgs c{};
        coords(p, c);
        SepArgs sa{};
        sa.X = gD;
        sa.out = gR;
        sa.H = p->H;
        sa.W = p->W;
        sa.h = p->h;
        sa.G = (int)p->sigmas.size();
        sa.fam = p->dSepFam;
        sa.M = p->M;
        sa.d_s = p->d_s;
        sa.sx = c.sx; sa.ox = c.ox; sa.sy = c.sy; sa.oy = c.oy;
        double* coefd = p->dVec + 7 * (size_t)kMaxCoefficients;
        double* gamma = p->dVec + 8 * (size_t)kMaxCoefficients;
        st = launch_sep_prep(a, p->dBeta, p->N, p->M, coefd, gamma, p->dSepCoef, p->stream);
        if (st) return st;
        sa.coefpf = reinterpret_cast<const float*>(p->dSepCoef + (size_t)(p->N + 1) * kSepCoefPad);
        st = launch_adjoint_r_sep_mma(sa, p->dSepFrag, p->stream);
        if (st) return st;
    } else if (gR && sep_form(p)) {
        // through the separable factors (E_n = c_n gD correlated with B_n)
        st = launch_adjoint_r_sep(p, a, gD, gR);
        if (st) return st;
    } else if (gR) {
        ContractArgs c{};
        c.X = gD;
        c.H = p->H;
        c.W = p->W;
        c.h = p->h;
        c.M = p->M;
        c.d_s = p->d_s;
        c.ped = 0.f;
        c.I = nullptr;
        c.out = gR;
        c.y_begin = 0;
        c.n_rows = p->H;
        coords(p, c);
        st = adjoint_filters(p->dF64, a, p->N, p->M, p->d_s, p->k, c.sx, c.sy, p->dFt32, p->stream);
        if (st) return st;
        st = build_f32_fragments(p->dFt32, p->M, p->k, p->dFragT32, p->stream);
        if (st) return st;
        c.NF = p->M;
        c.coef = nullptr;
        c.beta = nullptr;
        st = launch_contract_f32(c, p->dFragT32, (p->M + 15) / 16, p->stream);
        if (st) return st;
    }
    if (ga) st = run_adjoint_a(p, R, gD, ga);
    return st;
}

int svconv_loss_grad(svconv_plan* p, const float* D, const unsigned char* mask, float* gD,
                     double* loss) {
    if (!p || !D || !gD) return fail(SVCONV_EINVAL, "NULL argument");
    return launch_loss_grad(p, D, mask, gD, loss);
}

int svconv_normal_matrix(svconv_plan* p, const float* R, const unsigned char* mask, double* JtJ) {
    if (!p || !R || !JtJ) return fail(SVCONV_EINVAL, "NULL argument");
    return launch_normal_matrix(p, R, nullptr, mask, JtJ, nullptr);
}

int svconv_normal_equations(svconv_plan* p, const float* R, const float* I, const unsigned char* mask,
                            double* JtJ, double* rhs) {
    if (!p || !R || !I || !JtJ || !rhs) return fail(SVCONV_EINVAL, "NULL argument");
    return launch_normal_matrix(p, R, I, mask, JtJ, rhs);
}

int svconv_cholesky_factor(svconv_plan* p, double* A, int n) {
    if (!p || !A) return fail(SVCONV_EINVAL, "NULL argument");
    if (n <= 0 || n > kMaxCoefficients) return fail(SVCONV_EINVAL, "n out of range");
    return launch_cholesky(p, A, n);
}

int svconv_cholesky_solve(svconv_plan* p, const double* L, const double* rhs, double* x, int n) {
    if (!p || !L || !rhs || !x) return fail(SVCONV_EINVAL, "NULL argument");
    if (n <= 0 || n > kMaxCoefficients) return fail(SVCONV_EINVAL, "n out of range");
    return launch_cholesky_solve(p, L, rhs, x, n);
}

int svconv_gn_step(svconv_plan* p, const float* R, const float* I, const unsigned char* mask,
                   const double* L, double* a64, float* a32, float* D, double* host_stats) {
    if (!p || !R || !I || !L || !a64 || !a32 || !D) return fail(SVCONV_EINVAL, "NULL argument");
    if ((const void*)D == (const void*)R) return fail(SVCONV_EINVAL, "D aliases R");
    const int NK = p->N * p->M;          // kernel coefficients
    const int NM = NK + p->bg * p->M;    // plus the background polynomial
    double* ga = p->dVec;            // [NM]
    double* delta = p->dVec + NM;    // [NM]
    double* loss = p->dVec + 2 * NM; // scalar
    int st = launch_copy_a(p, a64, a32, NM);
    if (!st) st = run_forward(p, R, I, a32, D);
    if (!st && p->bg) st = launch_add_background(p, a32 + NK, D);
    if (!st) st = launch_loss_grad(p, D, mask, p->dGrad, loss);
    // the float64 adjoint: the split-precision one's error, through the
    // ill-conditioned normal matrix, keeps the steps from shrinking
    if (!st) st = launch_adjoint_a(p, R, p->dGrad, ga);
    if (!st && p->bg) st = launch_bg_grad(p, p->dGrad, ga + NK);
    if (!st) st = launch_scale(p, ga, 0.5, NM);
    if (!st) st = launch_cholesky_solve(p, L, ga, delta, NM);
    if (!st) st = launch_gn_update(p, delta, a64, a32, NM);
    if (st) return st;
    if (host_stats) {
        double stats[2] = {0.0, 0.0};
        st = hip_status(hipMemcpyAsync(&stats[0], loss, sizeof(double), hipMemcpyDeviceToHost, p->stream),
                        "copy loss");
        if (!st) st = hip_status(hipMemcpyAsync(&stats[1], p->dVec + 2 * NM + 1, sizeof(double),
                                                hipMemcpyDeviceToHost, p->stream), "copy step norm");
        if (!st) st = hip_status(hipStreamSynchronize(p->stream), "hipStreamSynchronize");
        if (st) return st;
        host_stats[0] = stats[0];
        host_stats[1] = stats[1];
    }
    return SVCONV_OK;
}

int svconv_ls_step(svconv_plan* p, const float* R, const float* I, const unsigned char* mask,
                   const double* A, const double* L, const double* rhs, double* a64, float* a32,
                   float* D, double* host_stats) {
    if (!p || !R || !I || !A || !L || !rhs || !a64 || !a32 || !D)
        return fail(SVCONV_EINVAL, "NULL argument");
    if ((const void*)D == (const void*)R) return fail(SVCONV_EINVAL, "D aliases R");
    const int NK = p->N * p->M;
    const int NM = NK + p->bg * p->M;
    double* g = p->dVec;             // [NM]
    double* delta = p->dVec + NM;    // [NM]
    double* loss = p->dVec + 2 * NM; // scalar
    // the residual and its loss at the current coefficients
    int st = launch_copy_a(p, a64, a32, NM);
    if (!st) st = run_forward(p, R, I, a32, D);
    if (!st && p->bg) st = launch_add_background(p, a32 + NK, D);
    if (!st) st = launch_loss_grad(p, D, mask, p->dGrad, loss);
    // J^T D = JtJ a - J^T I in float64, then the Newton step of the quadratic loss
    if (!st) st = launch_ls_grad(p, A, a64, rhs, g, NM);
    if (!st) st = launch_cholesky_solve(p, L, g, delta, NM);
    if (!st) st = launch_gn_update(p, delta, a64, a32, NM);
    if (st) return st;
    if (host_stats) {
        double stats[2] = {0.0, 0.0};
        st = hip_status(hipMemcpyAsync(stats, loss, 2 * sizeof(double), hipMemcpyDeviceToHost, p->stream),
                        "copy loss and step norm");
        if (!st) st = hip_status(hipStreamSynchronize(p->stream), "hipStreamSynchronize");
        if (st) return st;
        host_stats[0] = stats[0];
        host_stats[1] = stats[1];
    }
    return SVCONV_OK;
}

}  // extern "C"
