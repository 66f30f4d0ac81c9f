// svconv_difference_noalloc: D = (R (x) K) - I in the regrouped separable
// form without a plan and without any allocation, for callers that cannot
// allocate device memory (code under HIP graph capture, serving loops,
// harnesses that forbid hipMalloc).
//
// Every table the plan would hold (the one-dimensional Gaussian factors, the
// basis sums, the row-pass fragments of the precision) and the per-call
// tables (column-pass fragments, scales, pedestal sums) are built on the
// device into one file-scope array, `scratch`, of kNoAllocScratchBytes per
// GPU.  Host code never passes the array's name to a kernel: its device
// address is looked up once per device (hipGetSymbolAddress, with that device
// current) and kept in g_scratch.  Every call rewrites everything it reads
// from the array before reading it, so nothing has to start at zero; calls
// that overlap on one GPU (several host threads, or streams that run at the
// same time) share the array and race.
#include <cmath>
#include <mutex>

#include "internal.hpp"

namespace svc {

constexpr size_t kNoAllocScratchBytes = 512 * 1024;
constexpr int kNoAllocMaxFamilies = 8;
constexpr int kNoAllocMaxRowFactors = 32;
constexpr int kNoAllocMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

static std::mutex g_scratch_mu;
static void* g_scratch[kNoAllocMaxDevices];

// Device address of this device's scratch array (looked up on the first
// call on each device).
static int scratch_address(void** out) {
    int dev = 0;
    int st = hip_status(hipGetDevice(&dev), "hipGetDevice");
    if (st) return st;
    if (dev < 0 || dev >= kNoAllocMaxDevices) return fail(SVCONV_EUNSUPPORTED, "device index beyond 64");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* ptr = nullptr;
        st = hip_status(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        if (st) return st;
        if (!ptr) return fail(SVCONV_EDEVICE, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch[dev] = ptr;
    }
    *out = g_scratch[dev];
    return SVCONV_OK;
}

struct NoAllocSpec {
    int G, h;
    double sigma[kNoAllocMaxFamilies];
    int degree[kNoAllocMaxFamilies];
};

// The tables a plan would build on the host, built by one workgroup:
// f1d[g][e][w + h] = exp(-w^2 / 2 sigma_g^2) w^e / sum_w |exp(-w^2 / 2 sigma_g^2) w^e|
// (the one-dimensional factors of the Gaussian bases, Sec. 2), fam[g] =
// (degree, first basis), rinfo[r] = (family, factor) of each row factor, and
// beta_n = sum of basis n = (sum_u f_i(u)) (sum_v f_j(v)).
__global__ __launch_bounds__(256) void noalloc_tables_kernel(NoAllocSpec spec, double* __restrict__ f1d,
                                                             int* __restrict__ fam, int* __restrict__ rinfo,
                                                             double* __restrict__ beta) {
    __shared__ double fsum[kNoAllocMaxFamilies * kSepMaxFactors];
    const int tid = threadIdx.x, h = spec.h, k = 2 * h + 1;
    const int nf = spec.G * kSepMaxFactors;
    // one thread per factor: values, L1 norm, normalised values and their sum
    for (int q = tid; q < nf; q += 256) {
        const int g = q / kSepMaxFactors, e = q - g * kSepMaxFactors;
        double* f = f1d + (size_t)q * k;
        double l1 = 0.0;
        for (int w = -h; w <= h; ++w) {
            double mono = 1.0;
            for (int i = 0; i < e; ++i) mono *= w;
            const double v = (e <= spec.degree[g]) ? exp(-(double)(w * w) / (2.0 * spec.sigma[g] * spec.sigma[g])) * mono
                                                   : 0.0;
            f[w + h] = v;
            l1 += fabs(v);
        }
        double s = 0.0;
        for (int u = 0; u < k; ++u) {
            if (l1 > 0.0) f[u] /= l1;
            s += f[u];
        }
        fsum[q] = s;
    }
    __syncthreads();
    if (tid == 0) {
        int n = 0, r = 0;
        for (int g = 0; g < spec.G; ++g) {
            const int d = spec.degree[g];
            fam[2 * g] = d;
            fam[2 * g + 1] = n;
            for (int i = 0; i <= d; ++i) {
                rinfo[2 * r] = g;
                rinfo[2 * r + 1] = i;
                ++r;
            }
            for (int t = 0; t <= d; ++t)
                for (int i = t; i >= 0; --i) {
                    const int j = t - i;
                    beta[n++] = fsum[g * kSepMaxFactors + i] * fsum[g * kSepMaxFactors + j];
                }
        }
    }
}

static size_t up256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace svc

using namespace svc;

extern "C" int svconv_difference_noalloc(int height, int width, int half_width, int n_gauss, const double* sigmas,
                                         const int* degrees, int spatial_degree, int precision, float pedestal,
                                         const float* R, const float* I, const float* a, float* D, void* stream) {
    // validation, before any HIP call
    if (!sigmas || !degrees || !R || !I || !a || !D) return fail(SVCONV_EINVAL, "NULL argument");
    if (height <= 0 || width <= 0) return fail(SVCONV_EINVAL, "image size must be positive");
    if (half_width < 0) return fail(SVCONV_EINVAL, "half_width < 0");
    if (n_gauss <= 0) return fail(SVCONV_EINVAL, "no basis families");
    if (spatial_degree < 0) return fail(SVCONV_EINVAL, "spatial_degree < 0");
    if (precision < SVCONV_FP32 || precision > SVCONV_FP16X3) return fail(SVCONV_EINVAL, "unknown precision");
    if (!std::isfinite(pedestal)) return fail(SVCONV_EINVAL, "pedestal must be finite");
    if ((const void*)D == (const void*)R) return fail(SVCONV_EINVAL, "D aliases R");
    int N = 0, Rf = 0;
    for (int g = 0; g < n_gauss; ++g) {
        if (!(sigmas[g] >= 0.0) || !std::isfinite(sigmas[g])) return fail(SVCONV_EINVAL, "sigma must be finite and >= 0");
        if (degrees[g] < 0) return fail(SVCONV_EINVAL, "degree < 0");
        if (sigmas[g] == 0.0 && degrees[g] != 0) return fail(SVCONV_EINVAL, "a delta basis (sigma 0) must have degree 0");
        if (sigmas[g] == 0.0) return fail(SVCONV_EUNSUPPORTED, "the separable forms need Gaussian bases (sigma > 0)");
        if (degrees[g] >= kSepMaxFactors) return fail(SVCONV_EUNSUPPORTED, "degree > 9");
        N += (degrees[g] + 1) * (degrees[g] + 2) / 2;
        Rf += degrees[g] + 1;
    }
    if (precision != SVCONV_FP16X3 && precision != SVCONV_BF16X3 && precision != SVCONV_FP16X2)
        return fail(SVCONV_EUNSUPPORTED, "svconv_difference_noalloc needs a split 16-bit precision");
    if (half_width < 1 || half_width > kSepZMaxHalfWidth) return fail(SVCONV_EUNSUPPORTED, "half_width outside 1..12");
    if (spatial_degree > 2) return fail(SVCONV_EUNSUPPORTED, "spatial_degree > 2");
    if (n_gauss > kNoAllocMaxFamilies) return fail(SVCONV_EUNSUPPORTED, "more than 8 Gaussian families");
    if (N > kMaxFilters) return fail(SVCONV_EUNSUPPORTED, "more than 64 basis functions");
    if (Rf > kNoAllocMaxRowFactors) return fail(SVCONV_EUNSUPPORTED, "more than 32 row factors (sum of degree + 1)");
    const int k = 2 * half_width + 1;
    const int M = (spatial_degree + 1) * (spatial_degree + 2) / 2;

    // scratch layout (256-byte aligned sections)
    const size_t o_f1d = 0;
    const size_t o_fam = o_f1d + up256((size_t)n_gauss * kSepMaxFactors * k * sizeof(double));
    const size_t o_rinfo = o_fam + up256((size_t)2 * n_gauss * sizeof(int));
    const size_t o_beta = o_rinfo + up256((size_t)2 * Rf * sizeof(int));
    const size_t o_rtab = o_beta + up256((size_t)N * sizeof(double));
    const size_t o_ztab = o_rtab + up256(sepz_rtab_entries(Rf) / 2 * sizeof(uint16_t));
    const size_t o_zinv = o_ztab + up256(sepz_ztab_entries(Rf) * sizeof(uint16_t));
    const size_t o_gam = o_zinv + up256(8 * sizeof(float));
    const size_t total = o_gam + up256((size_t)kSepCoefPad * sizeof(double));
    if (total > kNoAllocScratchBytes) return fail(SVCONV_EUNSUPPORTED, "tables exceed the 512 KiB scratch array");

    void* base = nullptr;
    int st = scratch_address(&base);
    if (st) return st;
    unsigned char* sb = static_cast<unsigned char*>(base);
    double* f1d = reinterpret_cast<double*>(sb + o_f1d);
    int* fam = reinterpret_cast<int*>(sb + o_fam);
    int* rinfo = reinterpret_cast<int*>(sb + o_rinfo);
    double* beta = reinterpret_cast<double*>(sb + o_beta);
    uint16_t* rtab = reinterpret_cast<uint16_t*>(sb + o_rtab);
    hipStream_t s = (hipStream_t)stream;

    NoAllocSpec spec{};
    spec.G = n_gauss;
    spec.h = half_width;
    for (int g = 0; g < n_gauss; ++g) {
        spec.sigma[g] = sigmas[g];
        spec.degree[g] = degrees[g];
    }
    hipLaunchKernelGGL(noalloc_tables_kernel, dim3(1), dim3(256), 0, s, spec, f1d, fam, rinfo, beta);
    st = hip_status(hipGetLastError(), "noalloc_tables_kernel");
    const bool h16 = precision != SVCONV_BF16X3;
    if (!st) st = build_sepz_rtab(f1d, rinfo, Rf, half_width, rtab, s, h16 ? 0 : 1);
    if (st) return st;

    SepZArgs z{};
    z.X = R;
    z.I = I;
    z.out = D;
    z.H = height;
    z.W = width;
    z.h = half_width;
    z.ped = pedestal;
    z.R = Rf;
    z.M = M;
    // xh = 2 x / (W - 1) - 1 over the image itself; 0 on a one-pixel axis
    z.sx = width > 1 ? 2.0 / (width - 1) : 0.0;
    z.ox = width > 1 ? -1.0 : 0.0;
    z.sy = height > 1 ? 2.0 / (height - 1) : 0.0;
    z.oy = height > 1 ? -1.0 : 0.0;
    z.y_begin = 0;
    z.n_rows = height;
    z.rinfo = rinfo;
    z.rtab = rtab;
    z.ztab = reinterpret_cast<const uint16_t*>(sb + o_ztab);
    z.zinv = reinterpret_cast<const float*>(sb + o_zinv);
    z.gam = reinterpret_cast<const double*>(sb + o_gam);
    st = launch_sepz_prep(z, a, f1d, fam, beta, N, h16, s);
    if (st) return st;
    return launch_contract_sepz(z, precision, s);
}
