// Mixed-precision kernel product K V on 16-bit matrix cores (FP32 accumulation).
//
// Distances: the augmented contraction a_i . b_j (see prep.hip) carried out
// with every FP32 operand split exactly into three BF16 parts,
// v = v_h + v_m + v_l.  Per input dimension six part products are kept,
//     h.h + h.m + m.h + h.l + l.h + m.m,
// each exact in FP32; the dropped m.l + l.m + l.l terms are below 2^-24 of
// the product.  The exponent therefore keeps FP32-class accuracy while the
// contraction runs on 16x16x32 BF16 MFMA: (6 d + 6) slots per entry instead of
// the FP32 path's d + 2 slots at one eighth of the rate.  Slots:
//     6 per dimension r:  (2 xh_ir part) x (xh_jr part) as listed above
//     3:                  (c_i part) x 1        c_i = -|xh_i|^2
//     3:                  1 x (c_j part)        c_j = -|xh_j|^2
// The signal variance is not in the exponent: the tile holds K / sigma2 =
// exp2(S) <= 1 (up to rounding), and sigma2 multiplies the FP32 result.
//
// K V, three arithmetics:
//   BF16X1  K_h V_h with K_h = bf16(K), V_h = bf16(V): relative 2^-9.
//   BF16X3  K_h V_h + K_h V_l + K_l V_h, every part BF16 (K_l = bf16(K - K_h)):
//           relative ~2^-17.
//   F16X3   the same three products with FP16 parts.  K / sigma2 lies in
//           (0, 1], inside FP16's range; each V column is scaled by a power
//           of two that puts its largest magnitude in [2^14, 2^15) (exact),
//           and the scale is undone in the epilogue.  Parts carry 11
//           significant bits each: relative ~2^-22 per entry, with an
//           absolute floor of 2^-25 (of sigma2, resp. of the column's scaled
//           maximum) where a part falls below FP16's normal range.  The
//           remainder K - K_h takes one mixed FMA per entry that reads the
//           FP16 half straight from the packed dword (no conversion back).
// The column count is padded to a multiple of 16; the vector ALUs, which
// bound this kernel (exp2 and the splits), carry no column-dependent work.
//
// Lane layout: the transposed exponent tile leaves lane l holding K[i][j]
// for i = l % 16 and j = 4 (l / 16) + r of two 16-row j-tiles; those eight
// values are the A operand of the 16x16x32 K V MFMA, so V is packed with the
// matching permutation of its 32 rows:
//     element q of lane l in chunk T  <->  j = 32 T + 16 (q / 4) + 4 (l / 16) + q % 4.

#include "pkm_internal.h"

#include <algorithm>
#include <cmath>

namespace pkm {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));

__device__ inline void split3(float v, __bf16& h, __bf16& m, __bf16& l) {
    h = (__bf16)v;
    float r1 = v - (float)h;
    m = (__bf16)r1;
    float r2 = r1 - (float)m;
    l = (__bf16)r2;
}

// One thread per point: writes its 32 S6 slots on both sides.
__global__ void k_aug_bf16(const double* __restrict__ X, int64_t n, int64_t n_pad, int d,
                           int S6, const double* __restrict__ inv_l,
                           const double* __restrict__ mean,
                           __bf16* __restrict__ jsb, __bf16* __restrict__ isb) {
    int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i >= n_pad) return;
    const double cs = sqrt(0.5 * 1.4426950408889634);
    const int64_t t = i >> 4;
    const int rr = int(i & 15);
    auto addr = [&](int sl) {
        int s = sl >> 5, g = (sl & 31) >> 3, q = sl & 7;
        return ((t * S6 + s) * 64 + rr + 16 * g) * 8 + q;
    };
    const __bf16 one = (__bf16)1.0f, zero = (__bf16)0.0f;
    const int nslot = 32 * S6;
    for (int sl = 0; sl < nslot; ++sl) {
        jsb[addr(sl)] = zero;
        isb[addr(sl)] = zero;
    }
    double nrm = 0.0;
    float ci, cj;
    if (i < n) {
        for (int r = 0; r < d; ++r) {
            float xh = float((X[i * d + r] - mean[r]) * inv_l[r] * cs);
            nrm += double(xh) * double(xh);
            __bf16 ah, am, al, bh, bm, bl;
            split3(2.0f * xh, ah, am, al);
            split3(xh, bh, bm, bl);
            const __bf16 ia[6] = {ah, ah, am, ah, al, am};
            const __bf16 jb[6] = {bh, bm, bh, bl, bh, bm};
            for (int q = 0; q < 6; ++q) {
                isb[addr(6 * r + q)] = ia[q];
                jsb[addr(6 * r + q)] = jb[q];
            }
        }
        ci = float(-nrm);
        cj = ci;
    } else {
        ci = 0.0f;
        cj = -1.0e30f;
    }
    __bf16 h, m, l;
    split3(ci, h, m, l);
    const __bf16 cp[3] = {h, m, l};
    for (int q = 0; q < 3; ++q) {
        isb[addr(6 * d + q)] = cp[q];
        jsb[addr(6 * d + q)] = one;
    }
    split3(cj, h, m, l);
    const __bf16 dp[3] = {h, m, l};
    for (int q = 0; q < 3; ++q) {
        isb[addr(6 * d + 3 + q)] = one;
        jsb[addr(6 * d + 3 + q)] = dp[q];
    }
}

// Largest |V[:, c]| of each column as the bit pattern of a non-negative
// double (ordered like its value), max-reduced into colmax[c] (zeroed by the
// caller).  Thread t reads column t % k of rows t / k, t / k + L, ... with
// L = blockDim / k rows per pass, so a pass reads consecutive addresses.
__global__ void k_colmax(const double* __restrict__ V, int64_t ldv, int64_t n, int k,
                         unsigned long long* __restrict__ colmax) {
    __shared__ unsigned long long sm[kColmaxSlots];
    const int t = threadIdx.x;
    if (t < k) sm[t] = 0ull;
    __syncthreads();
    const int L = blockDim.x / k;
    if (t < L * k) {
        const int col = t % k;
        double m = 0.0;
#pragma unroll 4
        for (int64_t row = int64_t(blockIdx.x) * L + t / k; row < n; row += int64_t(gridDim.x) * L)
            m = fmax(m, fabs(V[row * ldv + col]));
        atomicMax(&sm[col], (unsigned long long)__double_as_longlong(m));
    }
    __syncthreads();
    if (t < k) atomicMax(&colmax[t], sm[t]);
}

__global__ void k_zero_slots(unsigned long long* __restrict__ slots) {
    slots[threadIdx.x] = 0ull;   // one block of kColmaxSlots threads
}

// Power-of-two exponent that takes column c's largest magnitude into
// [2^14, 2^15); 0 for an all-zero or non-finite column.
__device__ inline int col_shift(const unsigned long long* colmax, int c) {
    const double m = __longlong_as_double((long long)colmax[c]);
    if (!(m > 0.0) || !(m <= 1.7976931348623157e308)) return 0;
    return 14 - ilogb(m);
}

// Pack V (n x k FP64) for split NP: parts h (and l when NP == 3) in the
// permuted 32-row chunk order, plus the FP32 remainder columns.  With colmax
// (FP16 parts) each column is first scaled by 2^col_shift; otherwise the
// parts are BF16.  merge_last (FP16, at most 8 real columns in the last
// 16-column tile): that tile's part 0 carries the h parts of its columns in
// tile columns 0-7 and their l parts in tile columns 8-15 (part 1 unused).
//   vb[((T KT + qt) NPV + part) 64 + lane][q]
//   yr[((T KR + e) 4 + g) 8 + q]
__global__ void k_pack_v_bf16(const double* __restrict__ V, int64_t ldv, int64_t n, int k,
                              int nchunk, int KT, int KR, int NPV,
                              const unsigned long long* __restrict__ colmax, int merge_last,
                              __bf16* __restrict__ vb, float* __restrict__ yr) {
    int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    const int64_t per_chunk_v = int64_t(KT) * 64 * 8;   // one part
    const int64_t per_chunk_y = int64_t(KR) * 32;
    const int64_t tot = int64_t(nchunk) * (per_chunk_v + per_chunk_y);
    if (e >= tot) return;
    int64_t T = e / (per_chunk_v + per_chunk_y);
    int64_t w = e - T * (per_chunk_v + per_chunk_y);
    if (w < per_chunk_v) {
        int qt = int(w / 512);
        int rem = int(w % 512);
        int lane = rem >> 3, q = rem & 7;
        int g = lane >> 4;
        int64_t j = 32 * T + 16 * (q >> 2) + 4 * g + (q & 3);
        int col = 16 * qt + (lane & 15);
        int64_t base = ((T * KT + qt) * NPV) * 512 + lane * 8 + q;
        if (colmax && merge_last && qt == KT - 1) {
            const int c = 16 * qt + (lane & 7);
            const float v = (j < n && c < k) ? float(ldexp(V[j * ldv + c], col_shift(colmax, c))) : 0.0f;
            const _Float16 h = (_Float16)v;
            const _Float16 l = (_Float16)(v - (float)h);
            vb[base] = __builtin_bit_cast(__bf16, (lane & 8) ? l : h);
            vb[base + 512] = __builtin_bit_cast(__bf16, (_Float16)0.0f);
        } else if (colmax) {
            const float v = (j < n && col < k) ? float(ldexp(V[j * ldv + col], col_shift(colmax, col)))
                                               : 0.0f;
            const _Float16 h = (_Float16)v;
            vb[base] = __builtin_bit_cast(__bf16, h);
            if (NPV == 2) vb[base + 512] = __builtin_bit_cast(__bf16, (_Float16)(v - (float)h));
        } else {
            const float v = (j < n && col < k) ? float(V[j * ldv + col]) : 0.0f;
            const __bf16 h = (__bf16)v;
            vb[base] = h;
            if (NPV == 2) vb[base + 512] = (__bf16)(v - (float)h);
        }
    } else {
        int64_t w2 = w - per_chunk_v;
        int ee = int(w2 / 32);
        int rem = int(w2 % 32);
        int g = rem >> 3, q = rem & 7;
        int64_t j = 32 * T + 16 * (q >> 2) + 4 * g + (q & 3);
        int col = 16 * KT + ee;
        yr[((T * KR + ee) * 4 + g) * 8 + q] = (j < n && col < k) ? float(V[j * ldv + col]) : 0.0f;
    }
}

// Two floats -> one dword of two BF16 (round to nearest even).
__device__ inline uint32_t pack_bf16x2(float a, float b) {
    f32x2 v = {a, b};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));
}

// K (8 floats) -> K_h (and K_l = bf16(K - K_h) when NP == 3) as MFMA operands.
// The FP32 value of each rounded half is read back from the packed dword
// with one shift or mask instead of a second conversion.
template <int NP>
__device__ inline void split_k(const float (&kf)[8], bf16x8& kh, bf16x8& kl) {
    u32x4 h, l;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        const uint32_t w = pack_bf16x2(kf[2 * p], kf[2 * p + 1]);
        h[p] = w;
        if (NP == 3) {
            const float a = __builtin_bit_cast(float, w << 16);
            const float b = __builtin_bit_cast(float, w & 0xffff0000u);
            l[p] = pack_bf16x2(kf[2 * p] - a, kf[2 * p + 1] - b);
        }
    }
    kh = __builtin_bit_cast(bf16x8, h);
    if (NP == 3) kl = __builtin_bit_cast(bf16x8, l);
}

// Two floats -> one dword of two FP16 (round to nearest even).
__device__ inline uint32_t pack_f16x2(float a, float b) {
    f32x2 v = {a, b};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, f16x2));
}

// K (8 floats in (0, 1]) -> K_h = f16(K), K_l = f16(K - K_h).  The remainder
// is exact in FP32; v_fma_mix_f32 forms it as fma(-K_h, 1, K) with K_h read
// as the FP16 half (op_sel) of the packed dword.  The compiler keeps a
// conversion back to FP32 plus a subtraction for the same expression.
// (Measured and dropped: v_fma_mixlo_f16 / v_fma_mixhi_f16 writing the
// rounded remainders straight into the two halves of the K_l dword -- two
// ops per entry pair instead of three, bit-identical results -- ran 2-5 %
// slower at 65,536 points, k = 17 to 65.)
__device__ inline void split_k_f16(const float (&kf)[8], f16x8& kh, f16x8& kl) {
    u32x4 h, l;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        const uint32_t w = pack_f16x2(kf[2 * p], kf[2 * p + 1]);
        h[p] = w;
        float a, b;
        asm("v_fma_mix_f32 %0, -%1, 1.0, %2 op_sel_hi:[1,0,0]" : "=v"(a) : "v"(w), "v"(kf[2 * p]));
        asm("v_fma_mix_f32 %0, -%1, 1.0, %2 op_sel:[1,0,0] op_sel_hi:[1,0,0]"
            : "=v"(b) : "v"(w), "v"(kf[2 * p + 1]));
        l[p] = pack_f16x2(a, b);
    }
    kh = __builtin_bit_cast(f16x8, h);
    kl = __builtin_bit_cast(f16x8, l);
}

// Work-group: 4 waves x U i-tiles of 16 rows; loops over 32-row j-chunks of
// its j-split.  All k columns (padded to 16 KT) run on the matrix cores.
// NP: 1 = BF16X1, 3 = BF16X3, 4 = F16X3 (three FP16 products; colmax holds
// the column scales).  ML (F16X3 only): the last column tile is packed merged
// (h parts in tile columns 0-7, l parts in 8-15) and takes two MFMAs,
// (K_h + K_l) [V_h | V_l], instead of three; the epilogue adds column c + 8
// to column c.  The epilogue multiplies by sigma2 (and 2^-col_shift) and
// stores the k real columns of each row (row stride k; the padding columns
// are never written).
template <int S6, int KT, int U, int NP, bool ML>
__global__ __launch_bounds__(256) void k_mvm_bf16(
    const bf16x8* __restrict__ jsb, const bf16x8* __restrict__ isb,
    const bf16x8* __restrict__ vb, float* __restrict__ yout, int nchunk, int nrb, int jsplit,
    int chunks_per_split, int64_t split_stride, const unsigned long long* __restrict__ colmax,
    float s2, int kout) {
    constexpr int NPV = NP == 1 ? 1 : 2;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int b = blockIdx.x;
    const int xcd = b & 7, slot = b >> 3;
    const int group = 8 / jsplit;
    const int split = xcd % jsplit;
    const int rb = slot * group + xcd / jsplit;
    if (rb >= nrb) return;
    const int itile0 = (rb * 4 + wave) * U;
    const int g = lane >> 4;

    bf16x8 bi[U][S6];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
        for (int s = 0; s < S6; ++s) bi[u][s] = isb[(int64_t(itile0 + u) * S6 + s) * 64 + lane];

    f32x4 acc[U][KT];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
        for (int q = 0; q < KT; ++q) acc[u][q] = f32x4{0.f, 0.f, 0.f, 0.f};

    const int T0 = split * chunks_per_split;
    const int T1 = min(nchunk, T0 + chunks_per_split);
    const bf16x8* pa = jsb + int64_t(2 * T0) * S6 * 64 + lane;
    const bf16x8* pv = vb + int64_t(T0) * KT * NPV * 64 + lane;
    for (int T = T0; T < T1; ++T, pa += 2 * S6 * 64, pv += KT * NPV * 64) {
        bf16x8 a0[S6], a1[S6];
#pragma unroll
        for (int s = 0; s < S6; ++s) {
            a0[s] = pa[s * 64];
            a1[s] = pa[(S6 + s) * 64];
        }
        bf16x8 vv[KT][NPV];
#pragma unroll
        for (int qt = 0; qt < KT; ++qt)
#pragma unroll
            for (int pp = 0; pp < NPV; ++pp)
                if (!(ML && qt == KT - 1 && pp == 1)) vv[qt][pp] = pv[(qt * NPV + pp) * 64];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            f32x4 s0 = {0.f, 0.f, 0.f, 0.f}, s1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int s = 0; s < S6; ++s) {
                s0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0[s], bi[u][s], s0, 0, 0, 0);
                s1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1[s], bi[u][s], s1, 0, 0, 0);
            }
            float kf[8];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                kf[r] = __builtin_amdgcn_exp2f(s0[r]);
                kf[4 + r] = __builtin_amdgcn_exp2f(s1[r]);
            }
            if (NP == 4) {
                f16x8 kh, kl;
                split_k_f16(kf, kh, kl);
#pragma unroll
                for (int qt = 0; qt < KT; ++qt) {
                    const f16x8 vh = __builtin_bit_cast(f16x8, vv[qt][0]);
                    acc[u][qt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(kh, vh, acc[u][qt], 0, 0, 0);
                    if (!(ML && qt == KT - 1)) {
                        const f16x8 vl = __builtin_bit_cast(f16x8, vv[qt][NPV - 1]);
                        acc[u][qt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(kh, vl, acc[u][qt], 0, 0, 0);
                    }
                    acc[u][qt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(kl, vh, acc[u][qt], 0, 0, 0);
                }
            } else {
                bf16x8 kh, kl;
                split_k<NP>(kf, kh, kl);
#pragma unroll
                for (int qt = 0; qt < KT; ++qt) {
                    acc[u][qt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(kh, vv[qt][0], acc[u][qt], 0, 0, 0);
                    if (NP == 3) {
                        acc[u][qt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(kh, vv[qt][NPV - 1], acc[u][qt], 0, 0, 0);
                        acc[u][qt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(kl, vv[qt][0], acc[u][qt], 0, 0, 0);
                    }
                }
            }
        }
    }

    // undo the column scale first (exact while the result stays normal),
    // then one rounding for sigma2
    int sh[KT];
#pragma unroll
    for (int qt = 0; qt < KT; ++qt)
        sh[qt] = NP == 4 ? -col_shift(colmax, 16 * qt + (lane & ((ML && qt == KT - 1) ? 7 : 15))) : 0;
    float* yo = yout + int64_t(split) * split_stride;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int64_t row0 = int64_t(itile0 + u) * 16;
#pragma unroll
        for (int qt = 0; qt < KT; ++qt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int col = 16 * qt + (lane & 15);
                float v = acc[u][qt][r];
                bool keep = col < kout;
                if (ML && qt == KT - 1) {   // h half + l half (lanes l and l ^ 8)
                    v += __shfl_xor(v, 8);
                    keep = keep && (lane & 8) == 0;
                }
                const float a = NP == 4 ? ldexpf(v, sh[qt]) : v;
                if (keep) yo[(row0 + 4 * g + r) * kout + col] = a * s2;
            }
    }
}

void prepare_bf16(pkm_ctx* ctx) {
    Prepared& P = ctx->P();
    if (P.validb) return;
    PKM_REQUIRE(P.valid32, "internal: FP32 preparation must precede BF16 preparation");
    P.s6 = int(cdiv(6 * P.d + 6, 32));
    const int64_t ntiles = P.n_pad / 16;
    P.jsb.ensure(sizeof(__bf16) * ntiles * P.s6 * 64 * 8);
    P.isb.ensure(sizeof(__bf16) * ntiles * P.s6 * 64 * 8);
    const double* inv_l = ctx->scal.as<double>();
    const double* mean = inv_l + 64;
    k_aug_bf16<<<cdiv(P.n_pad, 128), 128, 0, ctx->stream>>>(
        P.X, P.n, P.n_pad, P.d, P.s6, inv_l, mean, P.jsb.as<__bf16>(), P.isb.as<__bf16>());
    PKM_CHECK_LAUNCH();
    P.validb = true;
}

constexpr int kBf16U = 4;   // i-tiles of 16 rows per wave

template <int S6, int NP, bool ML>
static void launch_bf16_s(int KT, dim3 grid, hipStream_t s, const bf16x8* js, const bf16x8* is,
                          const bf16x8* vb, float* y, int nchunk, int nrb, int jsplit, int cps,
                          int64_t stride, const unsigned long long* colmax, float s2, int kout) {
#define PKM_B_CASE(kt)                                                                         \
    if (KT == kt) {                                                                            \
        k_mvm_bf16<S6, kt, kBf16U, NP, ML><<<grid, 256, 0, s>>>(                               \
            js, is, vb, y, nchunk, nrb, jsplit, cps, stride, colmax, s2, kout);                \
        return;                                                                                \
    }
    PKM_B_CASE(1) PKM_B_CASE(2) PKM_B_CASE(3) PKM_B_CASE(4) PKM_B_CASE(5)
    PKM_B_CASE(6) PKM_B_CASE(7)
#undef PKM_B_CASE
    fail(PKM_ERR_UNSUPPORTED, "BF16 product: unsupported column count");
}

template <int NP, bool ML>
static void launch_bf16(int S6, int KT, dim3 grid, hipStream_t s, const bf16x8* js,
                        const bf16x8* is, const bf16x8* vb, float* y, int nchunk, int nrb,
                        int jsplit, int cps, int64_t stride, const unsigned long long* colmax,
                        float s2, int kout) {
#define PKM_S_CASE(s6)                                                                          \
    case s6:                                                                                    \
        launch_bf16_s<s6, NP, ML>(KT, grid, s, js, is, vb, y, nchunk, nrb, jsplit, cps, stride,     \
                              colmax, s2, kout);                                                \
        break;
    switch (S6) {
        PKM_S_CASE(1) PKM_S_CASE(2) PKM_S_CASE(3) PKM_S_CASE(4) PKM_S_CASE(5) PKM_S_CASE(6)
        PKM_S_CASE(7)
        default: fail(PKM_ERR_UNSUPPORTED, "BF16 product: d must be <= 36");
    }
#undef PKM_S_CASE
}

F32Out mvm_kbf16(pkm_ctx* ctx, int prec, int k, const double* V, int ldv) {
    Prepared& P = ctx->P();
    prepare_bf16(ctx);
    PKM_REQUIRE(k >= 1 && k <= kBf16MaxCols, "16-bit product: 1 <= k <= 112 columns per pass");
    const int NP = prec == PKM_F16X3 ? 4 : prec == PKM_BF16X3 ? 3 : 1;
    const int NPV = NP == 1 ? 1 : 2;
    const int KT = int(cdiv(k, 16));   // every column on the matrix cores
    const int KR = 0;
    const int nchunk = int(P.n_pad / 32);
    hipStream_t s = ctx->stream;
    const int64_t vb_elems = int64_t(nchunk) * KT * NPV * 512;
    const int64_t yr_elems = int64_t(nchunk) * KR * 32;
    const size_t vb_bytes = round_up(sizeof(__bf16) * std::max<int64_t>(vb_elems, 8), 256);
    const size_t yr_bytes = round_up(sizeof(float) * std::max<int64_t>(yr_elems, 4), 256);
    ctx->vbf.ensure(vb_bytes + yr_bytes);
    __bf16* vb = ctx->vbf.as<__bf16>();
    float* yrp = reinterpret_cast<float*>(reinterpret_cast<char*>(vb) + vb_bytes);
    unsigned long long* colmax = nullptr;
    if (NP == 4) {   // column scales for the FP16 parts (padded columns' slots stay 0)
        // the PCG direction update may have filled the slots for this V already
        const bool ready = ctx->colmax_src == V && ctx->colmax_k == k && ldv == k &&
                           ctx->colmax.bytes >= kColmaxSlots * sizeof(unsigned long long);
        ctx->colmax_src = nullptr;
        if (ready) {
            colmax = ctx->colmax.as<unsigned long long>();
        } else {
            // the slots start at zero: the previous product's k_finish32 cleared
            // them (cleared here after a fresh allocation or an interrupted call)
            if (ctx->colmax.bytes < kColmaxSlots * sizeof(unsigned long long))
                ctx->colmax_clean = false;
            ctx->colmax.ensure(kColmaxSlots * sizeof(unsigned long long));
            colmax = ctx->colmax.as<unsigned long long>();
            if (!ctx->colmax_clean) {   // a fill kernel, not a memset node (graph capture)
                k_zero_slots<<<1, kColmaxSlots, 0, s>>>(colmax);
                PKM_CHECK_LAUNCH();
            }
            ctx->colmax_clean = false;
            const int rows_per_pass = 256 / k;
            const int64_t blocks = std::min<int64_t>(512, cdiv(P.n, rows_per_pass));
            k_colmax<<<(unsigned)blocks, 256, 0, s>>>(V, ldv, P.n, k, colmax);
            PKM_CHECK_LAUNCH();
        }
    }
    const int64_t tot = int64_t(nchunk) * (int64_t(KT) * 512 + int64_t(KR) * 32);
    // FP16 parts: a last tile with at most 8 real columns is packed merged
    const bool ml = NP == 4 && k - 16 * (KT - 1) <= 8;
    k_pack_v_bf16<<<cdiv(tot, 256), 256, 0, s>>>(V, ldv, P.n, k, nchunk, KT, KR, NPV, colmax,
                                                  ml ? 1 : 0, vb, yrp);
    PKM_CHECK_LAUNCH();

    constexpr int U = kBf16U;
    const int64_t nrb = cdiv(P.n_pad, 64 * U);
    int jsplit = 1;
    while (jsplit < 8 && nrb * jsplit < 2048 && nchunk / (jsplit * 2) >= 8) jsplit <<= 1;
    const int cps = int(cdiv(nchunk, jsplit));
    const int group = 8 / jsplit;
    const int64_t nrb_pad = round_up(nrb, group);
    dim3 grid((unsigned)(nrb_pad * jsplit));
    const int64_t stride = P.n_pad * k;   // partial planes hold the k real columns
    ctx->y32.ensure(sizeof(float) * stride * jsplit);
    float* y = ctx->y32.as<float>();

    const hipEvent_t t0 = ctx->timing ? timing_start(ctx) : nullptr;
    const bf16x8* js = P.jsb.as<bf16x8>();
    const bf16x8* is = P.isb.as<bf16x8>();
    const bf16x8* vbv = reinterpret_cast<const bf16x8*>(vb);
    const float s2 = float(P.sigma2);
    if (NP == 1)
        launch_bf16<1, false>(P.s6, KT, grid, s, js, is, vbv, y, nchunk, int(nrb), jsplit, cps, stride,
                              colmax, s2, k);
    else if (NP == 3)
        launch_bf16<3, false>(P.s6, KT, grid, s, js, is, vbv, y, nchunk, int(nrb), jsplit, cps, stride,
                              colmax, s2, k);
    else if (ml)
        launch_bf16<4, true>(P.s6, KT, grid, s, js, is, vbv, y, nchunk, int(nrb), jsplit, cps, stride,
                             colmax, s2, k);
    else
        launch_bf16<4, false>(P.s6, KT, grid, s, js, is, vbv, y, nchunk, int(nrb), jsplit, cps, stride,
                              colmax, s2, k);
    PKM_CHECK_LAUNCH();
    if (t0) {
        const double pairs = double(P.n) * double(P.n);
        timing_stop(ctx, t0, prec, pairs, pairs * (2.0 * P.d + 2.0 * k));
    }
    return F32Out{y, jsplit, stride, k, colmax};
}

}  // namespace pkm
