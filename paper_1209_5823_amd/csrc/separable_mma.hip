// Separable form of the Gaussian-basis contraction on the matrix cores.
//
// The same factorisation as the float64 form (Sec. 2, Eq. 2 with separable
// Gaussian bases, B_n(u,v) = f_i(u) f_j(v)): a row pass per factor f_i, then
// a column pass per basis with f_j.  Each one-dimensional pass over a block
// of 16 outputs is a product with a banded Toeplitz matrix,
//   out[o] = sum_k F[o][k] x[k],   F[o][k] = f(o + 2h - k),  k in [0, 64),
// whose 64-long reduction covers the 16 + 2h samples the block needs (h <= 15
// gives at most 46).  The Toeplitz fragments depend only on the factor, so a
// per-plan table holds them in the lane order of v_mfma_f32_16x16x32_{f16,bf16}
// (lane l: index l mod 16, reduction entries 8 (l / 16) + 0..7 of each
// 32-long chunk), and the same values serve as the B operand of the row pass
// (n = output column) and the A operand of the column pass (m = output row).
//
// Precision: 16-bit inputs, float32 accumulation, with hi + lo splits
//   x = xh + xl, F = Fh + Fl (the taps rounded to nearest even; the data in
//   fp16 by the packed truncating conversion, the lo part holding the rest),
//   F x ~ Fh xh + Fh xl + Fl xh   (NT = 3; NT = 2 drops Fl xh),
// for R - s (scaled by 1/4 in fp16, as in the dense low-precision form) and for
// the row responses U between the passes.  The coefficient weighting c_n T_n
// and the sum over the bases run in float32 on the vector units; the pedestal
// restore s sum_m gamma_m P_m and the subtraction of I in float64.
//
// Workgroup: 8 waves, output tile 64 x 64.  LDS: the staged tile as hi / lo
// rows [96][120] (96 >= 64 + 2h rows; columns 0..111, zero past the halo) and,
// per round (one row factor), the row responses column-major as hi / lo
// [64][120] (rows 0..111; rows 96..111 stay zero).  A round: the products of
// the row pass (6 x 4 blocks of 16 x 16 per factor, spread over the waves; they
// read only the staged tile, so a wave starts them as soon as it has finished
// the previous round), a barrier, the responses written, a barrier, then the
// column pass, where wave w owns the 16-column block w mod 4 and the two
// 16-row blocks 2 (w / 4), 2 (w / 4) + 1 for every basis of the round, the
// products of basis j + 1 issued ahead of the epilogue of basis j.
#include "internal.hpp"
#include "sep_fold.hpp"

namespace svc {

typedef float smm_f4 __attribute__((ext_vector_type(4)));
typedef _Float16 smm_h8 __attribute__((ext_vector_type(8)));
typedef __bf16 smm_b8 __attribute__((ext_vector_type(8)));

constexpr int SM_NW = 8;
constexpr int SM_NT = 64 * SM_NW;
constexpr int SM_RB = 6;                 // row blocks of the row pass
constexpr int SM_XR = 16 * SM_RB;        // staged rows, >= 64 + 2h for h <= 15
constexpr int SM_XC = 112;               // staged columns the 64-long windows reach
constexpr int SM_UR = SM_XR + 16;        // row-response rows the column windows reach
constexpr int SM_P = 120;                // row / column pitch in 16-bit elements: 15 x 16 B (odd)
// One row factor per round keeps the LDS at 77 KB, two workgroups per CU, and
// the registers within four waves per SIMD (measured faster than three factors
// per round at one workgroup per CU).
constexpr int SM_SLOTS = 1;              // row factors per round
constexpr int SM_MINW = 4;               // waves per SIMD the registers allow
constexpr int SM_IB = SM_RB * 4 / SM_NW; // row-pass blocks per wave and round (3)
static_assert(SM_RB * 4 == SM_IB * SM_NW, "row-pass blocks must spread evenly over the waves");
constexpr int SM_FRAG = 2 * 2 * 64 * 8;  // 16-bit entries of one factor's table: [chunk][hi/lo][lane][8]
constexpr size_t SM_LDS = (size_t)(2 * SM_XR * SM_P + SM_SLOTS * 2 * 64 * SM_P) * sizeof(uint16_t);

__device__ __forceinline__ uint32_t smm_f2h(float x) {
    return (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)x);
}
__device__ __forceinline__ float smm_h2f(uint32_t b) { return (float)__builtin_bit_cast(_Float16, (uint16_t)b); }
__device__ __forceinline__ uint32_t smm_f2bf(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return u >> 16;
}
__device__ __forceinline__ float smm_bf2f(uint32_t b) { return __uint_as_float(b << 16); }

template <bool FP16>
__device__ __forceinline__ void smm_split(float x, uint32_t& hi, uint32_t& lo) {
    if (FP16) {
        hi = smm_f2h(x);
        lo = smm_f2h(x - smm_h2f(hi));
    } else {
        hi = smm_f2bf(x);
        lo = smm_f2bf(x - smm_bf2f(hi));
    }
}

// Two values split into packed hi and lo parts.  fp16: hi by the packed
// truncating conversion, lo the remainder x - hi (exact in float32) rounded to
// nearest even by one mixed-precision FMA per value (into the low, then the
// high half); bf16: rounded to nearest even one at a time.
template <bool FP16>
__device__ __forceinline__ void smm_split2(float x0, float x1, uint32_t& hi2, uint32_t& lo2) {
    if (FP16) {
        hi2 = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_pkrtz(x0, x1));
        uint32_t lo;
        asm("v_fma_mixlo_f16 %0, %1, -1.0, %2 op_sel_hi:[1,0,0]" : "=v"(lo) : "v"(hi2), "v"(x0));
        asm("v_fma_mixhi_f16 %0, %1, -1.0, %2 op_sel:[1,0,0] op_sel_hi:[1,0,0]" : "+v"(lo) : "v"(hi2), "v"(x1));
        lo2 = lo;
    } else {
        uint32_t h0, l0, h1, l1;
        smm_split<false>(x0, h0, l0);
        smm_split<false>(x1, h1, l1);
        hi2 = h0 | (h1 << 16);
        lo2 = l0 | (l1 << 16);
    }
}

// Sum over the 16 lanes of a DPP row, left in every lane of the row: mirror,
// half mirror, then the two quad swaps pair the lanes so that each step doubles
// the number of summed lanes.
template <int CTRL>
__device__ __forceinline__ float smm_dpp_mov(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xf, 0xf, false));
}
__device__ __forceinline__ float smm_row16_sum(float v) {
    v += smm_dpp_mov<0x140>(v);   // row_mirror: lane i + lane 15 - i
    v += smm_dpp_mov<0x141>(v);   // row_half_mirror: lane i + lane 7 - i within each half
    v += smm_dpp_mov<0x4e>(v);    // quad_perm [2, 3, 0, 1]
    v += smm_dpp_mov<0xb1>(v);    // quad_perm [1, 0, 3, 2]
    return v;
}

// bf16 hi by truncation (the low 16 bits of the float32 cleared), lo the
// remainder x - hi (exact in float32) rounded to nearest even: 2^-16 |x|, as
// the rounded split, at fewer instructions.
__device__ __forceinline__ void smm_split_bft(float x, uint32_t& hi, uint32_t& lo) {
    const uint32_t u = __float_as_uint(x) & 0xffff0000u;
    hi = u >> 16;
    lo = smm_f2bf(x - __uint_as_float(u));
}

template <bool FP16>
__device__ __forceinline__ smm_f4 smm_mfma(const uint4& a, const uint4& b, smm_f4 c) {
    if constexpr (FP16) {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(smm_h8, a),
                                                      __builtin_bit_cast(smm_h8, b), c, 0, 0, 0);
    } else {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(smm_b8, a),
                                                       __builtin_bit_cast(smm_b8, b), c, 0, 0, 0);
    }
}

// Toeplitz fragment tables of every factor, fp16 then bf16:
// frag[p][g][e][chunk][hi/lo][lane][t] = split(f_e^(g)(n + 2h - k)), n = lane mod 16,
// k = 32 chunk + 8 (lane / 16) + t, zero where n + 2h - k is outside [0, 2h].
__global__ void sep_mma_frag_kernel(const double* __restrict__ f1d, int G, int h,
                                    uint16_t* __restrict__ frag) {
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long per_factor = 2 * 64 * 8;             // [chunk][lane][t]
    const long total = 2L * G * kSepMaxFactors * per_factor;
    if (idx >= total) return;
    const int t = (int)(idx & 7);
    const int lane = (int)((idx >> 3) & 63);
    const int chunk = (int)((idx >> 9) & 1);
    const long ge = (idx >> 10) % ((long)G * kSepMaxFactors);
    const int p = (int)((idx >> 10) / ((long)G * kSepMaxFactors));
    const int k = 2 * h + 1;
    const int n = lane & 15, kk = 32 * chunk + 8 * (lane >> 4) + t;
    const int u = n + 2 * h - kk;
    const float v = (u >= 0 && u < k) ? (float)f1d[ge * k + u] : 0.f;
    uint32_t hi, lo;
    if (p == 0) smm_split<true>(v, hi, lo);
    else smm_split<false>(v, hi, lo);
    uint16_t* dst = frag + ((size_t)p * G * kSepMaxFactors + ge) * SM_FRAG;
    dst[((chunk * 2 + 0) * 64 + lane) * 8 + t] = (uint16_t)hi;
    dst[((chunk * 2 + 1) * 64 + lane) * 8 + t] = (uint16_t)lo;
}

int build_sep_mma_fragments(const double* f1d, int G, int h, uint16_t* frag, hipStream_t s) {
    const long total = 2L * G * kSepMaxFactors * 2 * 64 * 8;
    hipLaunchKernelGGL(sep_mma_frag_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, f1d,
                       G, h, frag);
    return hip_status(hipGetLastError(), "sep_mma_frag_kernel");
}

size_t sep_mma_frag_entries(int G) { return 2 * (size_t)G * kSepMaxFactors * SM_FRAG; }

// One factor's fragments for this lane: f[chunk][hi/lo].
__device__ __forceinline__ void smm_load_frag(const uint16_t* tab, int lane, uint4 (&f)[2][2]) {
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int hl = 0; hl < 2; ++hl)
            f[c][hl] = *reinterpret_cast<const uint4*>(tab + ((c * 2 + hl) * 64 + lane) * 8);
}

// ADJ: the adjoint in a instead of D.  The same passes give T_n(R - s) on the
// tile; the epilogue forms the moments sum_p G P_m T_n of the tile (per lane
// over its 8 pixels in powers of yh, over the 4 lanes of a column, weighted by
// the column's powers of xh, over the 16 columns of the wave) and adds them to
// one of kSepMomCopies copies of the sums (float64 atomics); slot N holds
// sum_p G P_m for the pedestal term.
// The adjoint instances at spatial degree above 3 hold the moments of
// (d + 1) powers across the column pass: they take 3 waves per SIMD (one
// workgroup per CU) so that their registers do not spill.
constexpr int smm_waves_per_simd(bool adj, int dsm) { return (adj && dsm > 3) ? 3 : SM_MINW; }

template <bool FP16, int NT, int DSM, bool ADJ = false>
__global__ __launch_bounds__(SM_NT, smm_waves_per_simd(ADJ, DSM)) void contract_sepmm_kernel(SepArgs a, const uint16_t* __restrict__ frag) {
    extern __shared__ uint4 smm_lds[];
    uint16_t* xs = reinterpret_cast<uint16_t*>(smm_lds);   // [2][SM_XR][SM_P]
    uint16_t* ut = xs + 2 * SM_XR * SM_P;                     // [SM_SLOTS][2][64][SM_P]

    const int h = a.h;
    const int RA = 64 + 2 * h, CA = 64 + 2 * h;
    const float xscale = FP16 ? 0.25f : 1.f;
    const double unscale = FP16 ? 4.0 : 1.0;
    const cptr<int> fam = as_const(a.fam);
    const uint16_t* ftab = frag + (FP16 ? 0 : (size_t)a.G * kSepMaxFactors * SM_FRAG);

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int t = sep_xcd_remap(blockIdx.x, a.n_tiles);
    const int X0 = (t % a.tiles_x) * 64;
    const int Y0 = a.y_begin + (t / a.tiles_x) * 64;
    const int y_end = min(a.H, a.y_begin + a.n_rows);

    // stage (R - s) * xscale as hi / lo, two columns per thread (32-bit LDS
    // writes); R = 0 outside the image; zero past the halo.  Every sample is
    // first loaded from a clamped, in-image address, none conditionally, so
    // that all loads are in flight together; the masks apply when storing.
    constexpr int SITER = (SM_XR * (SM_XC / 2) + SM_NT - 1) / SM_NT;
    float sv[SITER][2];
#pragma unroll
    for (int i = 0; i < SITER; ++i) {
        const int q = tid + i * SM_NT;
        const int r = q / (SM_XC / 2), c = 2 * (q - r * (SM_XC / 2));
        const float* src = a.X + (size_t)min(max(Y0 - h + r, 0), a.H - 1) * a.W;
#pragma unroll
        for (int e = 0; e < 2; ++e) sv[i][e] = src[min(max(X0 - h + c + e, 0), a.W - 1)];
    }
#pragma unroll
    for (int i = 0; i < SITER; ++i) {
        const int q = tid + i * SM_NT;
        if (q < SM_XR * (SM_XC / 2)) {
            const int r = q / (SM_XC / 2), c = 2 * (q - r * (SM_XC / 2));
            const int gy = Y0 - h + r;
            float v[2];
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const int gx = X0 - h + c + e;
                const float x = (gy >= 0 && gy < a.H && gx >= 0 && gx < a.W) ? sv[i][e] : 0.f;
                v[e] = (r < RA && c + e < CA) ? (x - a.ped) * xscale : 0.f;
            }
            uint32_t hi2, lo2;
            smm_split2<FP16>(v[0], v[1], hi2, lo2);
            *reinterpret_cast<uint32_t*>(xs + r * SM_P + c) = hi2;
            *reinterpret_cast<uint32_t*>(xs + (SM_XR + r) * SM_P + c) = lo2;
        }
    }
    // row-response rows SM_XR .. SM_UR - 1 are read by the column windows and never
    // written: zeroed once, 8 entries per write
    for (int q = tid; q < SM_SLOTS * 2 * 64 * ((SM_UR - SM_XR) / 8); q += SM_NT) {
        const int col = q / ((SM_UR - SM_XR) / 8), part = q - col * ((SM_UR - SM_XR) / 8);
        *reinterpret_cast<uint4*>(ut + col * SM_P + SM_XR + 8 * part) = make_uint4(0u, 0u, 0u, 0u);
    }

    // column-pass ownership: 16-column block cbB, row blocks rb0, rb0 + 1
    const int g4 = lane >> 4, j16 = lane & 15;
    const int cbB = w & 3, rb0 = 2 * (w >> 2);
    const int xl = 16 * cbB + j16;          // tile column of this lane's outputs
    const int x = X0 + xl;
    const double xh = a.sx * x + a.ox;
    float xpf[DSM + 1], yhf[2][4];
    xpf[0] = 1.f;
#pragma unroll
    for (int q = 1; q <= DSM; ++q) xpf[q] = xpf[q - 1] * (float)xh;
    float acc32[2][4];
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            // float32 arithmetic here: the float64 yh of the final pass is formed there
            yhf[b][e] = fmaf((float)a.sy, (float)(Y0 + 16 * (rb0 + b) + 4 * g4 + e), (float)a.oy);
            acc32[b][e] = 0.f;
        }
    const cptr<float> coefpf = as_const(a.coefpf);

    // adjoint in a: G at this lane's 8 output pixels (0 outside the image)
    float gq[2][4];
    double* mom = ADJ ? a.mom + (size_t)(blockIdx.x % kSepMomCopies) * (a.N + 1) * a.M : nullptr;
    auto flush = [&](int slot, float (&S)[DSM + 1]) {
#pragma unroll
        for (int q = 0; q <= DSM; ++q) {
            S[q] += __shfl_xor(S[q], 16);
            S[q] += __shfl_xor(S[q], 32);
        }
        // monomial m = tt (tt + 1) / 2 + jj is xh^(tt - jj) yh^jj; lane m keeps sum m
        float mine = 0.f;
        int m = 0;
#pragma unroll
        for (int tt = 0; tt <= DSM; ++tt)
#pragma unroll
            for (int jj = 0; jj <= tt; ++jj, ++m) {
                const float v = smm_row16_sum(xpf[tt - jj] * S[jj]);
                if (lane == m) mine = v;
            }
        if (lane < a.M) atomicAdd(mom + (size_t)slot * a.M + lane, (double)mine);
    };
    if constexpr (ADJ) {
        float S[DSM + 1];
#pragma unroll
        for (int q = 0; q <= DSM; ++q) S[q] = 0.f;
        // all eight loads first (clamped addresses), the masks after: a load
        // next to its mask is compiled into a branch of its own and waited for
        float gl[2][4];
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int y = Y0 + 16 * (rb0 + b) + 4 * g4 + e;
                gl[b][e] = a.I[(size_t)min(y, a.H - 1) * a.W + min(x, a.W - 1)];
            }
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int y = Y0 + 16 * (rb0 + b) + 4 * g4 + e;
                gq[b][e] = (x < a.W && y < y_end) ? gl[b][e] : 0.f;
                float tq = gq[b][e];
#pragma unroll
                for (int q = 0; q <= DSM; ++q) {
                    S[q] += tq;
                    tq *= yhf[b][e];
                }
            }
        flush(a.N, S);   // sum_p G P_m
    }

    __syncthreads();   // tile staged
    for (int g = 0; g < a.G; ++g) {
        const int deg = fam[2 * g], base = fam[2 * g + 1];
        const uint16_t* fg = ftab + (size_t)g * kSepMaxFactors * SM_FRAG;
        for (int i = 0; i <= deg; ++i) {
            // row pass: U_i[r][x'] in blocks of 16 rows x 16 columns, SM_IB per wave;
            // one accumulator per block, the products of a term issued across the
            // blocks so that dependent matrix-core operations are apart; only the
            // writes of the responses wait for every wave's previous column pass
            {
                uint4 tf[2][2];
                smm_load_frag(fg + (size_t)i * SM_FRAG, lane, tf);
                smm_f4 acc[SM_IB];
#pragma unroll
                for (int k = 0; k < SM_IB; ++k) acc[k] = smm_f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    uint4 dh[SM_IB], dl[SM_IB];
#pragma unroll
                    for (int k = 0; k < SM_IB; ++k) {
                        const int blk = w + k * SM_NW, rb = blk >> 2, cb = blk & 3;
                        const int off = (16 * rb + j16) * SM_P + 16 * cb + 32 * c + 8 * g4;
                        dh[k] = *reinterpret_cast<const uint4*>(xs + off);
                        dl[k] = *reinterpret_cast<const uint4*>(xs + SM_XR * SM_P + off);
                    }
#pragma unroll
                    for (int k = 0; k < SM_IB; ++k) acc[k] = smm_mfma<FP16>(dh[k], tf[c][0], acc[k]);
                    if (NT >= 2)
#pragma unroll
                        for (int k = 0; k < SM_IB; ++k) acc[k] = smm_mfma<FP16>(dl[k], tf[c][0], acc[k]);
                    if (NT >= 3)
#pragma unroll
                        for (int k = 0; k < SM_IB; ++k) acc[k] = smm_mfma<FP16>(dh[k], tf[c][1], acc[k]);
                }
                __syncthreads();   // previous round's row responses consumed
#pragma unroll
                for (int k = 0; k < SM_IB; ++k) {
                    const int blk = w + k * SM_NW, rb = blk >> 2, cb = blk & 3;
                    // lane (g4, j16) holds U at rows 16 rb + 4 g4 + e, column 16 cb + j16
                    const smm_f4 u = acc[k];
                    uint32_t hv[2], lv[2];
                    smm_split2<FP16>(u[0], u[1], hv[0], lv[0]);
                    smm_split2<FP16>(u[2], u[3], hv[1], lv[1]);
                    uint16_t* dst = ut + (size_t)(16 * cb + j16) * SM_P + 16 * rb + 4 * g4;
                    *reinterpret_cast<uint2*>(dst) = make_uint2(hv[0], hv[1]);
                    *reinterpret_cast<uint2*>(dst + 64 * SM_P) = make_uint2(lv[0], lv[1]);
                }
            }
            __syncthreads();
            // column pass: T_n = f_j (x)_y U_i on this wave's two blocks, then D += c_n T_n
            uint4 ub[2][2][2];   // [block][chunk][hi/lo]
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int ch = 0; ch < 2; ++ch)
#pragma unroll
                    for (int hl = 0; hl < 2; ++hl)
                        ub[b][ch][hl] = *reinterpret_cast<const uint4*>(
                            ut + ((size_t)hl * 64 + xl) * SM_P + 16 * (rb0 + b) + 32 * ch + 8 * g4);
            // the products of basis j + 1 are issued ahead of the epilogue of basis j
            // (two accumulator sets, one accumulator per block over both chunks)
            const int nb = deg - i + 1;
            auto products = [&](int j, smm_f4 (&acc)[2]) {
                uint4 tf[2][2];
                smm_load_frag(fg + (size_t)j * SM_FRAG, lane, tf);
#pragma unroll
                for (int b = 0; b < 2; ++b) acc[b] = smm_f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int ch = 0; ch < 2; ++ch)
#pragma unroll
                    for (int b = 0; b < 2; ++b) acc[b] = smm_mfma<FP16>(tf[ch][0], ub[b][ch][0], acc[b]);
                if (NT >= 2)
#pragma unroll
                    for (int ch = 0; ch < 2; ++ch)
#pragma unroll
                        for (int b = 0; b < 2; ++b) acc[b] = smm_mfma<FP16>(tf[ch][0], ub[b][ch][1], acc[b]);
                if (NT >= 3)
#pragma unroll
                    for (int ch = 0; ch < 2; ++ch)
#pragma unroll
                        for (int b = 0; b < 2; ++b) acc[b] = smm_mfma<FP16>(tf[ch][1], ub[b][ch][0], acc[b]);
            };
            auto epilogue = [&](int j, const smm_f4 (&acc)[2]) {
                const int n = base + (i + j) * (i + j + 1) / 2 + j;
                if constexpr (ADJ) {
                    float S[DSM + 1];
#pragma unroll
                    for (int q = 0; q <= DSM; ++q) S[q] = 0.f;
#pragma unroll
                    for (int b = 0; b < 2; ++b)
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            float tq = gq[b][e] * acc[b][e];
#pragma unroll
                            for (int q = 0; q <= DSM; ++q) {
                                S[q] += tq;
                                tq *= yhf[b][e];
                            }
                        }
                    flush(n, S);
                    return;
                }
                float cy[DSM + 1];
#pragma unroll
                for (int q = 0; q <= DSM; ++q) cy[q] = 0.f;
                {
                    const cptr<float> cn_ = coefpf + (size_t)n * kSepCoefPad;
                    int m = 0;
#pragma unroll
                    for (int tt = 0; tt <= DSM; ++tt) {
#pragma unroll
                        for (int ie = tt; ie >= 0; --ie) cy[tt - ie] = fmaf(cn_[m + tt - ie], xpf[ie], cy[tt - ie]);
                        m += tt + 1;
                    }
                }
#pragma unroll
                for (int b = 0; b < 2; ++b)
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        float cn = cy[DSM];
#pragma unroll
                        for (int q = DSM - 1; q >= 0; --q) cn = fmaf(cn, yhf[b][e], cy[q]);
                        acc32[b][e] = fmaf(cn, acc[b][e], acc32[b][e]);
                    }
            };
            smm_f4 accA[2], accB[2];
            products(0, accA);
            for (int j = 0;;) {
                if (j + 1 < nb) products(j + 1, accB);
                epilogue(j, accA);
                if (++j >= nb) break;
                if (j + 1 < nb) products(j + 1, accA);
                epilogue(j, accB);
                if (++j >= nb) break;
            }
        }
    }
    if (!ADJ && x < a.W) {
        // pedestal restore s sum_m gamma_m P_m (float64), then D = sum_n c_n T_n - I
        double xpow[DSM + 1];
        xpow[0] = 1.0;
#pragma unroll
        for (int q = 1; q <= DSM; ++q) xpow[q] = xpow[q - 1] * xh;
        double cy[DSM + 1];
        coef_in_x<DSM>(as_const(a.gammap), xpow, cy);
        // I at this lane's pixels, all requested at once from clamped addresses
        // (without I, R stands in for the loads)
        float iv[2][4];
        {
            const float* ip = a.I ? a.I : a.X;
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    iv[b][e] = ip[(size_t)min(Y0 + 16 * (rb0 + b) + 4 * g4 + e, a.H - 1) * a.W + x];
        }
        const bool has_i = a.I != nullptr;
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int y = Y0 + 16 * (rb0 + b) + 4 * g4 + e;
                if (y < y_end) {
                    const double yh = a.sy * y + a.oy;
                    double pg = cy[DSM];
#pragma unroll
                    for (int q = DSM - 1; q >= 0; --q) pg = fma(pg, yh, cy[q]);
                    const size_t idx = (size_t)y * a.W + x;
                    a.out[idx] = (float)(fma((double)acc32[b][e], unscale, (double)a.ped * pg) -
                                         (has_i ? (double)iv[b][e] : 0.0));
                }
            }
    }
}

template <bool FP16, int NT>
static int launch_sepmm_p(const SepArgs& a, const uint16_t* frag, hipStream_t s) {
    if (a.d_s <= 2)
        hipLaunchKernelGGL((contract_sepmm_kernel<FP16, NT, 2>), dim3(a.n_tiles), dim3(SM_NT), SM_LDS, s, a, frag);
    else
        hipLaunchKernelGGL((contract_sepmm_kernel<FP16, NT, kMaxSpatialDegree>), dim3(a.n_tiles), dim3(SM_NT),
                           SM_LDS, s, a, frag);
    return hip_status(hipGetLastError(), "contract_sepmm_kernel");
}

int launch_contract_sep_mma(SepArgs a, const uint16_t* frag, int precision, hipStream_t s) {
    if (a.h < 1 || a.h > 15) return fail(SVCONV_EUNSUPPORTED, "separable form needs 1 <= half-width <= 15");
    if (a.tout) return fail(SVCONV_EINVAL, "the matrix-core separable kernel has no T-only mode");
    a.tiles_x = (a.W + 63) / 64;
    a.n_tiles = a.tiles_x * ((a.n_rows + 63) / 64);
    switch (precision) {
        case SVCONV_FP16X3: return launch_sepmm_p<true, 3>(a, frag, s);
        case SVCONV_BF16X3: return launch_sepmm_p<false, 3>(a, frag, s);
        case SVCONV_FP16X2: return launch_sepmm_p<true, 2>(a, frag, s);
        default: return fail(SVCONV_EINVAL, "no matrix-core separable kernel for this precision");
    }
}


__global__ void sep_mom_zero(double* __restrict__ mom, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) mom[i] = 0.0;
}

// ga[n][m] = unscale sum_c mom[c][n][m] + s beta_n sum_c mom[c][N][m] (copies in order)
__global__ void sep_mom_final(const double* __restrict__ mom, int N, int M, double unscale,
                              const double* __restrict__ beta, float ped, double* __restrict__ ga) {
    const int nm = blockIdx.x * blockDim.x + threadIdx.x;
    if (nm >= N * M) return;
    const int n = nm / M, m = nm - n * M;
    const size_t stride = (size_t)(N + 1) * M;
    double s = 0.0, gp = 0.0;
    for (int c = 0; c < kSepMomCopies; ++c) {
        s += mom[c * stride + nm];
        gp += mom[c * stride + (size_t)N * M + m];
    }
    ga[nm] = unscale * s + (double)ped * beta[n] * gp;
}

template <bool FP16>
static int launch_asepmm_p(const SepArgs& a, const uint16_t* frag, hipStream_t s) {
    if (a.d_s <= 2)
        hipLaunchKernelGGL((contract_sepmm_kernel<FP16, 3, 2, true>), dim3(a.n_tiles), dim3(SM_NT), SM_LDS, s, a, frag);
    else if (a.d_s == 3)
        hipLaunchKernelGGL((contract_sepmm_kernel<FP16, 3, 3, true>), dim3(a.n_tiles), dim3(SM_NT), SM_LDS, s, a, frag);
    else if (a.d_s <= 4)
        hipLaunchKernelGGL((contract_sepmm_kernel<FP16, 3, 4, true>), dim3(a.n_tiles), dim3(SM_NT), SM_LDS, s, a, frag);
    else
        hipLaunchKernelGGL((contract_sepmm_kernel<FP16, 3, kMaxSpatialDegree, true>), dim3(a.n_tiles), dim3(SM_NT),
                           SM_LDS, s, a, frag);
    return hip_status(hipGetLastError(), "contract_sepmm_kernel (adjoint in a)");
}

int launch_adjoint_a_sep_mma(SepArgs a, const uint16_t* frag, int precision, const double* beta,
                             double* ga, hipStream_t s) {
    if (a.h < 1 || a.h > 15) return fail(SVCONV_EUNSUPPORTED, "separable form needs 1 <= half-width <= 15");
    if (a.M > 64) return fail(SVCONV_EUNSUPPORTED, "matrix-core adjoint in a needs M <= 64");
    a.tiles_x = (a.W + 63) / 64;
    a.n_tiles = a.tiles_x * ((a.n_rows + 63) / 64);
    a.tout = nullptr;
    const int n_mom = kSepMomCopies * (a.N + 1) * a.M;
    hipLaunchKernelGGL(sep_mom_zero, dim3((n_mom + 255) / 256), dim3(256), 0, s, a.mom, n_mom);
    int st = hip_status(hipGetLastError(), "sep_mom_zero");
    if (st) return st;
    const bool fp16 = precision == SVCONV_FP16X3;
    st = fp16 ? launch_asepmm_p<true>(a, frag, s) : launch_asepmm_p<false>(a, frag, s);
    if (st) return st;
    const int NM = a.N * a.M;
    hipLaunchKernelGGL(sep_mom_final, dim3((NM + 255) / 256), dim3(256), 0, s, a.mom, a.N, a.M,
                       fp16 ? 4.0 : 1.0, beta, a.ped, ga);
    return hip_status(hipGetLastError(), "sep_mom_final");
}

// ------------------------------------------------------- adjoint in R ----
//
//   dL/dR(q) = sum_n sum_{u,v} B_n[u,v] E_n(q + (u,v)),   E_n = c_n G
//
// (the correlation of Sec. 2's forward with B_n = f_i(u) f_j(v)), on the same
// Toeplitz fragments: a correlation is the convolution with the mirrored
// factor, f_e(-w) = (-1)^e f_e(w), so the sign (-1)^j goes into E_n and (-1)^i
// into CE_i.  Per 64 x 64 output tile and basis n = (i, j): E_n on the tile and
// its halo ((64 + 2h)^2, c_n in float32 from the padded float coefficients, G
// held in registers for the whole tile), split into bf16 hi + lo column-major
// in LDS; the column pass CE_i += f_j (x)_y E_n accumulates over the bases of
// row factor i in the matrix-core accumulators (4 x 6 blocks, 3 per wave); then
// CE_i is split row-major into LDS and the row pass dR += f_i (x)_x CE_i
// accumulates over all rounds (4 x 4 blocks, 2 per wave).  bf16 keeps the
// float32 range of c_n G (hi by truncation, lo rounded); three products per
// pass as in the forward.
constexpr int SA_NI = 9;                  // E entries per thread and basis, as row pairs
static_assert(SM_XR * (SM_XR / 2) == SA_NI * SM_NT, "E row pairs must spread evenly over the threads");
constexpr int SA_CYP = 8;                 // Cy entries per staged column (spatial degree <= 7)
constexpr size_t SA_LDS = SM_LDS + (size_t)SM_XR * SA_CYP * sizeof(float);   // 78 KB: two workgroups per CU
static_assert(kMaxSpatialDegree + 1 <= SA_CYP, "Cy table too narrow");

template <int DSM>
__global__ __launch_bounds__(SM_NT, SM_MINW) void adjoint_r_sepmm_kernel(SepArgs a, const uint16_t* __restrict__ frag) {
    extern __shared__ uint4 smm_lds[];
    uint16_t* et = reinterpret_cast<uint16_t*>(smm_lds);   // [2][SM_XR columns][SM_P]: E_n, rows contiguous
    uint16_t* ce = et + 2 * SM_XR * SM_P;                    // [2][64 rows][SM_P]: CE_i, columns contiguous
    float* cyt = reinterpret_cast<float*>(ce + 2 * 64 * SM_P);  // [SM_XR][SA_CYP]: Cy of the basis per column

    const int h = a.h;
    const int CA = 64 + 2 * h;
    const cptr<int> fam = as_const(a.fam);
    const cptr<float> coefpf = as_const(a.coefpf);
    const uint16_t* ftab = frag + (size_t)a.G * kSepMaxFactors * SM_FRAG;   // bf16 tables

    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int g4 = lane >> 4, j16 = lane & 15;
    const int t = sep_xcd_remap(blockIdx.x, a.n_tiles);
    const int X0 = (t % a.tiles_x) * 64, Y0 = (t / a.tiles_x) * 64;
    const float sxf = (float)a.sx, oxf = (float)a.ox, syf = (float)a.sy, oyf = (float)a.oy;

    // E rows SM_XR .. SM_UR - 1 and CE columns SM_XR .. SM_UR - 1 are read by the
    // last windows and never written: zeroed once, 8 entries per write
    for (int q = tid; q < 2 * SM_XR * 2; q += SM_NT)
        *reinterpret_cast<uint4*>(et + (q >> 1) * SM_P + SM_XR + 8 * (q & 1)) = make_uint4(0u, 0u, 0u, 0u);
    for (int q = tid; q < 2 * 64 * 2; q += SM_NT)
        *reinterpret_cast<uint4*>(ce + (q >> 1) * SM_P + SM_XR + 8 * (q & 1)) = make_uint4(0u, 0u, 0u, 0u);
    // G on the staged region (row pairs q = tid + k SM_NT: column q / 48, rows
    // 2 (q mod 48) + 0, 1); zero outside the image and past the halo
    float gv[SA_NI][2];
#pragma unroll
    for (int k = 0; k < SA_NI; ++k) {
        const int q = tid + k * SM_NT, xq = q / (SM_XR / 2), pr = q - xq * (SM_XR / 2);
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int yq = 2 * pr + e, gx = X0 - h + xq, gy = Y0 - h + yq;
            gv[k][e] = a.X[(size_t)min(max(gy, 0), a.H - 1) * a.W + min(max(gx, 0), a.W - 1)];
        }
    }
    // (loaded from clamped addresses above so that no load is conditional;
    // masked here)
#pragma unroll
    for (int k = 0; k < SA_NI; ++k) {
        const int q = tid + k * SM_NT, xq = q / (SM_XR / 2), pr = q - xq * (SM_XR / 2);
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int yq = 2 * pr + e, gx = X0 - h + xq, gy = Y0 - h + yq;
            if (!(xq < CA && yq < CA && gx >= 0 && gx < a.W && gy >= 0 && gy < a.H)) gv[k][e] = 0.f;
        }
    }
    smm_f4 accR[2];   // dR blocks w and w + 8 of the 4 x 4 output blocks
#pragma unroll
    for (int k = 0; k < 2; ++k) accR[k] = smm_f4{0.f, 0.f, 0.f, 0.f};

    for (int g = 0; g < a.G; ++g) {
        const int deg = fam[2 * g], base = fam[2 * g + 1];
        const uint16_t* fg = ftab + (size_t)g * kSepMaxFactors * SM_FRAG;
        for (int i = 0; i <= deg; ++i) {
            smm_f4 accC[SM_IB];   // CE_i blocks w, w + 8, w + 16 of the 4 x 6 blocks
#pragma unroll
            for (int k = 0; k < SM_IB; ++k) accC[k] = smm_f4{0.f, 0.f, 0.f, 0.f};
            for (int j = 0; j + i <= deg; ++j) {
                const int n = base + (i + j) * (i + j + 1) / 2 + j;
                const float sgn = (j & 1) ? -1.f : 1.f;
                __syncthreads();   // previous basis' E and Cy consumed
                // c_n(x, y) = sum_q Cy[q](x) yh^q with Cy[q] = sum_{t >= q} c[t (t + 1) / 2 + q] xh^(t - q)
                // (the monomial x^(t-q) y^q), per staged column into LDS
                {
                    const cptr<float> cn_ = coefpf + (size_t)n * kSepCoefPad;
                    for (int e = tid; e < SM_XR * (DSM + 1); e += SM_NT) {
                        const int xq = e / (DSM + 1), qq = e - xq * (DSM + 1);
                        const float xh = fmaf(sxf, (float)(X0 - h + xq), oxf);
                        float cy = 0.f;
                        for (int tt = DSM; tt >= qq; --tt) cy = fmaf(cy, xh, cn_[tt * (tt + 1) / 2 + qq]);
                        cyt[xq * SA_CYP + qq] = cy;
                    }
                }
                __syncthreads();
                // E_n = (-1)^j c_n G
#pragma unroll
                for (int k = 0; k < SA_NI; ++k) {
                    const int q = tid + k * SM_NT, xq = q / (SM_XR / 2), pr = q - xq * (SM_XR / 2);
                    float cy[DSM + 1];
#pragma unroll
                    for (int qq = 0; qq <= DSM; ++qq) cy[qq] = cyt[xq * SA_CYP + qq];
                    float v[2];
#pragma unroll
                    for (int e = 0; e < 2; ++e) {
                        const float yh = fmaf(syf, (float)(Y0 - h + 2 * pr + e), oyf);
                        float cn = cy[DSM];
#pragma unroll
                        for (int qq = DSM - 1; qq >= 0; --qq) cn = fmaf(cn, yh, cy[qq]);
                        v[e] = sgn * cn * gv[k][e];
                    }
                    uint32_t h0, l0, h1, l1;
                    smm_split_bft(v[0], h0, l0);
                    smm_split_bft(v[1], h1, l1);
                    *reinterpret_cast<uint32_t*>(et + xq * SM_P + 2 * pr) = h0 | (h1 << 16);
                    *reinterpret_cast<uint32_t*>(et + (SM_XR + xq) * SM_P + 2 * pr) = l0 | (l1 << 16);
                }
                __syncthreads();
                // column pass: block (rb, cb) = (blk mod 4, blk / 4), A = taps of f_j,
                // B = E at columns 16 cb + (lane mod 16), rows 16 rb + [0, 64)
                uint4 tf[2][2];
                smm_load_frag(fg + (size_t)j * SM_FRAG, lane, tf);
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    uint4 eh[SM_IB], el[SM_IB];
#pragma unroll
                    for (int k = 0; k < SM_IB; ++k) {
                        const int blk = w + k * SM_NW, rb = blk & 3, cb = blk >> 2;
                        const int off = (16 * cb + j16) * SM_P + 16 * rb + 32 * c + 8 * g4;
                        eh[k] = *reinterpret_cast<const uint4*>(et + off);
                        el[k] = *reinterpret_cast<const uint4*>(et + SM_XR * SM_P + off);
                    }
#pragma unroll
                    for (int k = 0; k < SM_IB; ++k) accC[k] = smm_mfma<false>(tf[c][0], eh[k], accC[k]);
#pragma unroll
                    for (int k = 0; k < SM_IB; ++k) accC[k] = smm_mfma<false>(tf[c][0], el[k], accC[k]);
#pragma unroll
                    for (int k = 0; k < SM_IB; ++k) accC[k] = smm_mfma<false>(tf[c][1], eh[k], accC[k]);
                }
            }
            // CE_i (sign (-1)^i) split row-major: lane (g4, j16) holds rows
            // 16 rb + 4 g4 + e, column 16 cb + j16
            __syncthreads();   // previous round's CE consumed
            {
                const float sgi = (i & 1) ? -1.f : 1.f;
#pragma unroll
                for (int k = 0; k < SM_IB; ++k) {
                    const int blk = w + k * SM_NW, rb = blk & 3, cb = blk >> 2;
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        uint32_t hi, lo;
                        smm_split_bft(sgi * accC[k][e], hi, lo);
                        const int off = (16 * rb + 4 * g4 + e) * SM_P + 16 * cb + j16;
                        ce[off] = (uint16_t)hi;
                        ce[64 * SM_P + off] = (uint16_t)lo;
                    }
                }
            }
            __syncthreads();
            // row pass: block (rb, cb) = (blk / 4, blk mod 4), A = CE at rows
            // 16 rb + (lane mod 16), columns 16 cb + [0, 64), B = taps of f_i
            {
                uint4 tf[2][2];
                smm_load_frag(fg + (size_t)i * SM_FRAG, lane, tf);
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    uint4 chh[2], chl[2];
#pragma unroll
                    for (int k = 0; k < 2; ++k) {
                        const int blk = w + k * SM_NW, rb = blk >> 2, cb = blk & 3;
                        const int off = (16 * rb + j16) * SM_P + 16 * cb + 32 * c + 8 * g4;
                        chh[k] = *reinterpret_cast<const uint4*>(ce + off);
                        chl[k] = *reinterpret_cast<const uint4*>(ce + 64 * SM_P + off);
                    }
#pragma unroll
                    for (int k = 0; k < 2; ++k) accR[k] = smm_mfma<false>(chh[k], tf[c][0], accR[k]);
#pragma unroll
                    for (int k = 0; k < 2; ++k) accR[k] = smm_mfma<false>(chl[k], tf[c][0], accR[k]);
#pragma unroll
                    for (int k = 0; k < 2; ++k) accR[k] = smm_mfma<false>(chh[k], tf[c][1], accR[k]);
                }
            }
        }
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int blk = w + k * SM_NW, rb = blk >> 2, cb = blk & 3;
        const int x = X0 + 16 * cb + j16;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int y = Y0 + 16 * rb + 4 * g4 + e;
            if (x < a.W && y < a.H) a.out[(size_t)y * a.W + x] = accR[k][e];
        }
    }
}

int launch_adjoint_r_sep_mma(SepArgs a, const uint16_t* frag, hipStream_t s) {
    if (a.h < 1 || a.h > 15) return fail(SVCONV_EUNSUPPORTED, "separable form needs 1 <= half-width <= 15");
    a.tiles_x = (a.W + 63) / 64;
    a.n_tiles = a.tiles_x * ((a.H + 63) / 64);
    if (a.d_s <= 2)
        hipLaunchKernelGGL(adjoint_r_sepmm_kernel<2>, dim3(a.n_tiles), dim3(SM_NT), SA_LDS, s, a, frag);
    else if (a.d_s == 3)
        hipLaunchKernelGGL(adjoint_r_sepmm_kernel<3>, dim3(a.n_tiles), dim3(SM_NT), SA_LDS, s, a, frag);
    else if (a.d_s <= 4)
        hipLaunchKernelGGL(adjoint_r_sepmm_kernel<4>, dim3(a.n_tiles), dim3(SM_NT), SA_LDS, s, a, frag);
    else
        hipLaunchKernelGGL(adjoint_r_sepmm_kernel<kMaxSpatialDegree>, dim3(a.n_tiles), dim3(SM_NT), SA_LDS, s, a, frag);
    return hip_status(hipGetLastError(), "adjoint_r_sepmm_kernel");
}

}  // namespace svc
