// Batched PCG: many independent GP problems (own X, theta, lambda, n, d and
// preconditioner) solved together, every PCG phase one launch for all of
// them (Algorithm 1 per problem and per right-hand-side column).
//
// Layout: the problems' rows are packed one after another, each padded to a
// multiple of 256 rows; every FP64 vector (x, r, z, p, K_y p, b) is one
// packed n_total x k block, and a per-256-row-block table names the problem.
// Padding rows stay zero throughout.
//
// Kernel product: one work-queue launch per input-dimension class (the
// augmented length fixes the MFMA shape).  Work items are (problem, row
// block, column-range split) triples ordered largest problem first; every
// work-group pulls items with an atomic counter until the list is
// exhausted, so uneven problems balance across the chip and no work-group
// ever waits on another.  A problem is split over its columns j (up to 8
// ranges, partial sums added in a fixed order afterwards) when its row
// blocks alone would leave the chip idle, which keeps the last, largest
// problems fast once the others have converged.  Problems whose columns
// have all converged are skipped.
//
// The launch shape (i-tiles per wave) is chosen per class by a small
// autotuner that times the candidates on the first call and caches the
// winner in memory and, if PKM_TUNE_CACHE names a file, in that JSON file.

#include "pkm_internal.h"

#include <cstdio>
#include <cstdlib>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <fstream>
#include <map>
#include <mutex>
#include <cstring>
#include <sstream>
#include <string>
#include <tuple>

namespace pkm {

struct BDesc {
    int64_t row0;          // packed row offset
    int64_t n;             // rows of this problem
    int64_t tile0;         // row0 / 16
    int64_t ntiles;        // n_pad / 16 of its own prepared operands
    const float* jside;
    const float* iside;
    const double* psi;     // preconditioner (NULL: none)
    const double* dinv;
    int m;
    int pad;
    double lambda;
    int64_t partoff;       // phase-1 partial sums offset (doubles)
    int64_t toff;          // padded T offset (doubles)
    int64_t rpc;           // phase-1 rows per chunk
    int nchunk;
    int mpad;
    const void* jsb;       // FP16x3 products: BF16 operand slots (prep.hip / mvm_bf16.hip)
    const void* isb;
    double sigma2;
};

struct BCol {
    double rz, alpha, beta, bnorm, rec, tru, rr;
    int32_t active, status, parked, restart;
    int64_t iters;
    double ref;   // true relative residual at the last replacement
    double eta;   // refinement mode (restart at replacement, inner target eta * ref)
};

struct BFlags {
    int32_t live, pending, broke, pad;
};

__device__ inline bool bstep(const BCol& s) { return s.active && !s.parked; }

// ---------------------------------------------------------------------------
// work-queue FP32 kernel product (same inner loop as the single-problem one)
// ---------------------------------------------------------------------------
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <int S4, int KT, int KR, int U>
__global__ __launch_bounds__(256) void k_bmvm_f32(const BDesc* __restrict__ desc,
                                                  const int4* __restrict__ items, int nitems,
                                                  int* __restrict__ counter,
                                                  const int* __restrict__ live,
                                                  const int* __restrict__ use64,
                                                  const float* __restrict__ vs,
                                                  float* __restrict__ ybase, int64_t split_stride) {
    constexpr int KP = 16 * KT + KR;
    __shared__ int sh_item;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int g = lane >> 4;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) sh_item = atomicAdd(counter, 1);
        __syncthreads();
        const int it = sh_item;
        if (it >= nitems) return;
        const int4 item = items[it];   // problem, row block, split, splits
        if (!live[item.x] || use64[item.x]) continue;
        const BDesc D = desc[item.x];
        const int64_t tps = (D.ntiles + item.w - 1) / item.w;
        const int64_t t_beg = item.z * tps;
        const int64_t t_end = min(D.ntiles, t_beg + tps);
        float* __restrict__ yout = ybase + item.z * split_stride;
        const int64_t itile0 = (int64_t(item.y) * 4 + wave) * U;   // local tile
        float bi[U][S4];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int s = 0; s < S4; ++s) bi[u][s] = D.iside[((itile0 + u) * 64 + lane) * S4 + s];
        f32x4 acc[U][KT > 0 ? KT : 1];
        float racc[U][KR > 0 ? KR : 1];
#pragma unroll
        for (int u = 0; u < U; ++u) {
#pragma unroll
            for (int q = 0; q < (KT > 0 ? KT : 1); ++q) acc[u][q] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int e = 0; e < (KR > 0 ? KR : 1); ++e) racc[u][e] = 0.f;
        }
        // one j-tile's operands, two register sets in turn (as k_mvm_f32)
        struct Tile {
            float aj[S4];
            f32x4 vv[KT > 0 ? KT : 1];
            f32x4 yr[KR > 0 ? KR : 1];
        };
        auto load = [&](int64_t t, Tile& T) {
#pragma unroll
            for (int s = 0; s < S4; ++s) T.aj[s] = D.jside[(t * 64 + lane) * S4 + s];
            const float* vt = vs + (D.tile0 + t) * 16 * KP;
#pragma unroll
            for (int q = 0; q < KT; ++q) T.vv[q] = *reinterpret_cast<const f32x4*>(vt + q * 256 + lane * 4);
#pragma unroll
            for (int e = 0; e < KR; ++e)
                T.yr[e] = *reinterpret_cast<const f32x4*>(vt + KT * 256 + e * 16 + g * 4);
        };
        auto step = [&](const Tile& T) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                f32x4 st = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int s = 0; s < S4; ++s)
                    st = __builtin_amdgcn_mfma_f32_16x16x4f32(T.aj[s], bi[u][s], st, 0, 0, 0);
                float kv[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) kv[r] = __builtin_amdgcn_exp2f(st[r]);
#pragma unroll
                for (int q = 0; q < KT; ++q)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        acc[u][q] = __builtin_amdgcn_mfma_f32_16x16x4f32(kv[r], T.vv[q][r], acc[u][q], 0, 0, 0);
#pragma unroll
                for (int e = 0; e < KR; ++e)
                    racc[u][e] += kv[0] * T.yr[e][0] + kv[1] * T.yr[e][1] + kv[2] * T.yr[e][2] +
                                  kv[3] * T.yr[e][3];
            }
        };
        if (t_beg < t_end) {
            Tile A, B;
            load(t_beg, A);
            for (int64_t t = t_beg; t < t_end; t += 2) {
                load(min(t + 1, t_end - 1), B);
                step(A);
                if (t + 1 >= t_end) break;
                load(min(t + 2, t_end - 1), A);
                step(B);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t row0 = D.row0 + (itile0 + u) * 16;
#pragma unroll
            for (int q = 0; q < KT; ++q)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    yout[(row0 + 4 * g + r) * KP + 16 * q + (lane & 15)] = acc[u][q][r];
#pragma unroll
            for (int e = 0; e < KR; ++e) {
                float v = racc[u][e];
                v += __shfl_xor(v, 16);
                v += __shfl_xor(v, 32);
                if (g == 0) yout[(row0 + (lane & 15)) * KP + 16 * KT + e] = v;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// work-queue FP16x3 kernel product (inner loop as k_mvm_bf16 with NP = 4):
// BF16-split exponent on BF16 MFMA, K / sigma2 and the power-of-two-scaled
// V columns (per problem) as FP16 parts on FP16 MFMA, FP32 accumulation.
// Items as k_bmvm_f32: (problem, row block of 64 U rows, split, splits); a
// split covers a contiguous range of the problem's 32-row j-chunks.  ML: the
// last column tile is packed merged ([V_h | V_l], at most 8 columns).
// Partial planes hold the k real columns of each row (row stride k).
// ---------------------------------------------------------------------------
typedef __bf16 bbf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 bf16h8 __attribute__((ext_vector_type(8)));
typedef _Float16 bf16h2 __attribute__((ext_vector_type(2)));
typedef float bf32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t bu32x4 __attribute__((ext_vector_type(4)));

__device__ inline uint32_t bpack_f16x2(float a, float b) {
    bf32x2 v = {a, b};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16h2));
}

// K -> K_h = f16(K), K_l = f16(K - K_h); the remainder by one mixed FMA
// reading the FP16 half of the packed dword (v_fma_mix_f32)
__device__ inline void bsplit_k_f16(const float (&kf)[8], bf16h8& kh, bf16h8& kl) {
    bu32x4 h, l;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        const uint32_t w = bpack_f16x2(kf[2 * p], kf[2 * p + 1]);
        h[p] = w;
        float a, b;
        asm("v_fma_mix_f32 %0, -%1, 1.0, %2 op_sel_hi:[1,0,0]" : "=v"(a) : "v"(w), "v"(kf[2 * p]));
        asm("v_fma_mix_f32 %0, -%1, 1.0, %2 op_sel:[1,0,0] op_sel_hi:[1,0,0]"
            : "=v"(b) : "v"(w), "v"(kf[2 * p + 1]));
        l[p] = bpack_f16x2(a, b);
    }
    kh = __builtin_bit_cast(bf16h8, h);
    kl = __builtin_bit_cast(bf16h8, l);
}

// power-of-two exponent taking a column's largest magnitude into [2^14, 2^15)
__device__ inline int bcol_shift(const unsigned long long* colmax, int c) {
    const double m = __longlong_as_double((long long)colmax[c]);
    if (!(m > 0.0) || !(m <= 1.7976931348623157e308)) return 0;
    return 14 - ilogb(m);
}

template <int S6, int KT, int U, bool ML>
__global__ __launch_bounds__(256) void k_bmvm_f16(const BDesc* __restrict__ desc,
                                                  const int4* __restrict__ items, int nitems,
                                                  int* __restrict__ counter,
                                                  const int* __restrict__ live,
                                                  const int* __restrict__ use64,
                                                  const bbf16x8* __restrict__ vb,
                                                  const unsigned long long* __restrict__ colmax,
                                                  int k, float* __restrict__ ybase,
                                                  int64_t split_stride) {
    constexpr int NPV = 2;
    __shared__ int sh_item;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int g = lane >> 4;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) sh_item = atomicAdd(counter, 1);
        __syncthreads();
        const int it = sh_item;
        if (it >= nitems) return;
        const int4 item = items[it];   // problem, row block, split, splits
        if (!live[item.x] || use64[item.x]) continue;
        const BDesc D = desc[item.x];
        const bbf16x8* __restrict__ jsb = static_cast<const bbf16x8*>(D.jsb);
        const bbf16x8* __restrict__ isb = static_cast<const bbf16x8*>(D.isb);
        const int64_t nch = D.ntiles / 2;   // 32-row j-chunks of this problem
        const int64_t cps = (nch + item.w - 1) / item.w;
        const int64_t c_beg = item.z * cps;
        const int64_t c_end = min(nch, c_beg + cps);
        float* __restrict__ yout = ybase + item.z * split_stride;
        const int64_t itile0 = (int64_t(item.y) * 4 + wave) * U;   // local i-tile
        bbf16x8 bi[U][S6];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int s = 0; s < S6; ++s) bi[u][s] = isb[((itile0 + u) * S6 + s) * 64 + lane];
        f32x4 acc[U][KT];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int q = 0; q < KT; ++q) acc[u][q] = f32x4{0.f, 0.f, 0.f, 0.f};
        const bbf16x8* pa = jsb + 2 * c_beg * S6 * 64 + lane;
        const bbf16x8* pv = vb + (D.tile0 / 2 + c_beg) * KT * NPV * 64 + lane;
        for (int64_t T = c_beg; T < c_end; ++T, pa += 2 * S6 * 64, pv += KT * NPV * 64) {
            bbf16x8 a0[S6], a1[S6];
#pragma unroll
            for (int s = 0; s < S6; ++s) {
                a0[s] = pa[s * 64];
                a1[s] = pa[(S6 + s) * 64];
            }
            bbf16x8 vv[KT][NPV];
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
                bf16h8 kh, kl;
                bsplit_k_f16(kf, kh, kl);
#pragma unroll
                for (int qt = 0; qt < KT; ++qt) {
                    const bf16h8 vh = __builtin_bit_cast(bf16h8, vv[qt][0]);
                    acc[u][qt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(kh, vh, acc[u][qt], 0, 0, 0);
                    if (!(ML && qt == KT - 1)) {
                        const bf16h8 vl = __builtin_bit_cast(bf16h8, vv[qt][1]);
                        acc[u][qt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(kh, vl, acc[u][qt], 0, 0, 0);
                    }
                    acc[u][qt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(kl, vh, acc[u][qt], 0, 0, 0);
                }
            }
        }
        const unsigned long long* cm = colmax + int64_t(item.x) * k;
        int sh[KT];
#pragma unroll
        for (int qt = 0; qt < KT; ++qt) {
            const int c = 16 * qt + (lane & ((ML && qt == KT - 1) ? 7 : 15));
            sh[qt] = c < k ? -bcol_shift(cm, c) : 0;
        }
        const float s2 = float(D.sigma2);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t row0 = D.row0 + (itile0 + u) * 16;
#pragma unroll
            for (int qt = 0; qt < KT; ++qt)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int col = 16 * qt + (lane & 15);
                    float v = acc[u][qt][r];
                    bool keep = col < k;
                    if (ML && qt == KT - 1) {   // h half + l half (lanes l and l ^ 8)
                        v += __shfl_xor(v, 8);
                        keep = keep && (lane & 8) == 0;
                    }
                    if (keep) yout[(row0 + 4 * g + r) * k + col] = ldexpf(v, sh[qt]) * s2;
                }
        }
    }
}

// colmax[b k + c] = largest |V[row, c]| over problem b's rows (bit pattern of a
// non-negative double), one work-group per 256-row block; colmax zeroed first
__global__ __launch_bounds__(256) void k_bcolmax(const double* __restrict__ V, int k,
                                                 const int* __restrict__ rbprob,
                                                 unsigned long long* __restrict__ colmax) {
    __shared__ unsigned long long sm[64];
    const int t = threadIdx.x;
    if (t < k) sm[t] = 0ull;
    __syncthreads();
    const int L = 256 / k;
    const int64_t r0 = int64_t(blockIdx.x) * 256;
    if (t < L * k) {
        const int col = t % k;
        double m = 0.0;
        for (int rr = t / k; rr < 256; rr += L) m = fmax(m, fabs(V[(r0 + rr) * k + col]));
        atomicMax(&sm[col], (unsigned long long)__double_as_longlong(m));
    }
    __syncthreads();
    if (t < k) atomicMax(&colmax[int64_t(rbprob[blockIdx.x]) * k + t], sm[t]);
}

// packed p (n_total x k FP64) -> FP16 parts in the permuted 32-row chunk
// order of k_bmvm_f16 (global chunk index), each problem's columns scaled by
// its own powers of two; rows past a problem's n pack as zero
__global__ void k_bpack_v16(const double* __restrict__ V, int64_t nchunk, int k, int KT, int ml,
                            const int* __restrict__ rbprob, const BDesc* __restrict__ desc,
                            const unsigned long long* __restrict__ colmax,
                            __bf16* __restrict__ vb) {
    const int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    const int64_t per_chunk = int64_t(KT) * 512;
    if (e >= nchunk * per_chunk) return;
    const int64_t T = e / per_chunk;
    const int w = int(e - T * per_chunk);
    const int qt = w / 512, rem = w % 512;
    const int lane = rem >> 3, q = rem & 7;
    const int64_t j = 32 * T + 16 * (q >> 2) + 4 * (lane >> 4) + (q & 3);
    const int b = rbprob[j >> 8];
    const bool valid = j - desc[b].row0 < desc[b].n;
    const unsigned long long* cm = colmax + int64_t(b) * k;
    const int64_t base = ((T * KT + qt) * 2) * 512 + lane * 8 + q;
    if (ml && qt == KT - 1) {
        const int c = 16 * qt + (lane & 7);
        const float v = (valid && c < k) ? float(ldexp(V[j * k + c], bcol_shift(cm, c))) : 0.0f;
        const _Float16 h = (_Float16)v;
        const _Float16 l = (_Float16)(v - (float)h);
        vb[base] = __builtin_bit_cast(__bf16, (lane & 8) ? l : h);
        vb[base + 512] = __builtin_bit_cast(__bf16, (_Float16)0.0f);
    } else {
        const int c = 16 * qt + (lane & 15);
        const float v = (valid && c < k) ? float(ldexp(V[j * k + c], bcol_shift(cm, c))) : 0.0f;
        const _Float16 h = (_Float16)v;
        vb[base] = __builtin_bit_cast(__bf16, h);
        vb[base + 512] = __builtin_bit_cast(__bf16, (_Float16)(v - (float)h));
    }
}

// p (packed FP64, n_total x k) -> MFMA lane-order tiles (global tile index)
__global__ void k_bpack_v32(const double* __restrict__ V, int64_t ntot, int k, int KT, int KR,
                            float* __restrict__ vs) {
    const int KP = 16 * KT + KR;
    int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    const int64_t tot = (ntot / 16) * 16 * KP;
    if (e >= tot) return;
    int64_t t = e / (16 * KP);
    int w = int(e - t * 16 * KP);
    int64_t row;
    int col;
    if (w < KT * 256) {
        int q = w >> 8, rem = w & 255;
        int l = rem >> 2, r = rem & 3;
        row = 16 * t + 4 * (l >> 4) + r;
        col = 16 * q + (l & 15);
    } else {
        int w2 = w - KT * 256;
        row = 16 * t + (w2 & 15);
        col = 16 * KT + (w2 >> 4);
    }
    vs[e] = col < k ? float(V[row * k + col]) : 0.f;
}

// Ap = (sum of the problem's split partials) + lambda_b p on valid rows
// (padding rows stay zero); splits are added in order, in FP64
__global__ void k_bfinish32(const float* __restrict__ y, int64_t split_stride, int kp,
                            int64_t ntot, int k, const int* __restrict__ rbprob,
                            const BDesc* __restrict__ desc, const int* __restrict__ nsplit,
                            const double* __restrict__ p, double* __restrict__ Ap) {
    int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (e >= ntot * k) return;
    const int64_t row = e / k;
    const int c = int(e - row * k);
    const int b = rbprob[row >> 8];
    const BDesc& D = desc[b];
    if (row - D.row0 >= D.n) {
        Ap[e] = 0.0;
        return;
    }
    double acc = 0.0;
    for (int q = 0; q < nsplit[b]; ++q) acc += double(y[q * split_stride + row * kp + c]);
    Ap[e] = acc + D.lambda * p[e];
}

// ---------------------------------------------------------------------------
// per-problem reductions and recurrences
// ---------------------------------------------------------------------------
// part[rb][c] = sum over the 256 rows of row-block rb of u o v (k <= 256)
__global__ __launch_bounds__(256) void k_bdot_part(const double* __restrict__ u,
                                                   const double* __restrict__ v, int k,
                                                   double* __restrict__ part) {
    __shared__ double sh[256];
    const int per = 256 / k;
    const int T = per * k;
    const int64_t beg = int64_t(blockIdx.x) * 256 * k, end = beg + int64_t(256) * k;
    double acc = 0.0;
    if (threadIdx.x < T)
        for (int64_t e = beg + threadIdx.x; e < end; e += T) acc = fma(u[e], v[e], acc);
    sh[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x < k) {
        double s = 0.0;
        for (int q = 0; q < per; ++q) s += sh[threadIdx.x + q * k];
        part[int64_t(blockIdx.x) * k + threadIdx.x] = s;
    }
}

__device__ inline double bsum(const double* part, const int* rbrange, int b, int k, int c) {
    double s = 0.0;
    for (int rb = rbrange[b]; rb < rbrange[b + 1]; ++rb) s += part[int64_t(rb) * k + c];
    return s;
}

__global__ void k_binit(const double* __restrict__ pbb, const double* __restrict__ prz,
                        const int* __restrict__ rbrange, int P, int k, BCol* __restrict__ st) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= P * k) return;
    const int b = e / k, c = e - b * k;
    const double bb = bsum(pbb, rbrange, b, k, c);
    BCol s{};
    s.bnorm = sqrt(bb);
    s.rz = bsum(prz, rbrange, b, k, c);
    s.active = bb > 0.0 ? 1 : 0;
    s.status = PKM_COL_CONVERGED;
    s.rec = s.tru = s.ref = bb > 0.0 ? 1.0 : 0.0;
    if (!isfinite(bb) || !isfinite(s.rz) || (s.active && !(s.rz > 0.0))) {
        s.active = 0;
        s.status = PKM_COL_BREAKDOWN;
    }
    st[e] = s;
}

// Also clears the status accumulators that k_brr fills later in the same
// step (the previous step's copies to the host were queued before this
// kernel; no kernel in between reads them).
__global__ void k_balpha(const double* __restrict__ ppap, const int* __restrict__ rbrange, int P,
                         int k, BCol* __restrict__ st, BFlags* __restrict__ fl,
                         int* __restrict__ live_prob, int* __restrict__ broke_prob,
                         int* __restrict__ act_prob) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e == 0) *fl = BFlags{};
    if (e < P) {
        live_prob[e] = 0;
        broke_prob[e] = 0;
        act_prob[e] = 0;
    }
    if (e >= P * k) return;
    const int b = e / k, c = e - b * k;
    BCol s = st[e];
    if (bstep(s)) {
        const double pap = bsum(ppap, rbrange, b, k, c);
        if (!(pap > 0.0) || !isfinite(pap)) {
            s.active = 0;
            s.status = PKM_COL_BREAKDOWN;
            s.alpha = 0.0;
        } else {
            s.alpha = s.rz / pap;
            s.iters += 1;
        }
    } else {
        s.alpha = 0.0;
    }
    st[e] = s;
}

__device__ inline const BCol& col_of(const BCol* st, const int* rbprob, int64_t e, int k) {
    const int64_t row = e / k;
    return st[int64_t(rbprob[row >> 8]) * k + (e - row * k)];
}

__global__ void k_bupdate_xr(int64_t tot, int k, const int* __restrict__ rbprob,
                             const BCol* __restrict__ st, const double* __restrict__ p,
                             const double* __restrict__ Ap, double* __restrict__ x,
                             double* __restrict__ r) {
    int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (e >= tot) return;
    const double a = col_of(st, rbprob, e, k).alpha;
    if (a != 0.0) {
        x[e] = fma(a, p[e], x[e]);
        r[e] = fma(-a, Ap[e], r[e]);
    }
}

__global__ void k_brr(const double* __restrict__ prr, const int* __restrict__ rbrange, int P,
                      int k, double tol, BCol* __restrict__ st, BFlags* __restrict__ fl,
                      int* __restrict__ live_prob, int* __restrict__ broke_prob,
                      int* __restrict__ act_prob) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= P * k) return;
    const int b = e / k, c = e - b * k;
    BCol s = st[e];
    const double rr = bsum(prr, rbrange, b, k, c);
    s.rr = rr;
    s.rec = s.bnorm > 0.0 ? sqrt(rr) / s.bnorm : 0.0;
    if (s.active && !isfinite(rr)) {
        s.active = 0;
        s.status = PKM_COL_BREAKDOWN;
    }
    if (bstep(s) && s.rec <= fmax(tol, s.eta * s.ref)) s.parked = 1;
    if (s.active) {
        atomicAdd(&fl->live, 1);
        atomicOr(&act_prob[b], 1);
        if (!s.parked) {
            atomicAdd(&fl->pending, 1);
            atomicOr(&live_prob[b], 1);
        }
    }
    if (s.status == PKM_COL_BREAKDOWN) {
        atomicAdd(&fl->broke, 1);
        atomicAdd(&broke_prob[b], 1);
    }
    st[e] = s;
}

__global__ void k_btrue_res(int64_t tot, int k, const int* __restrict__ rbprob,
                            const BCol* __restrict__ st, const double* __restrict__ b,
                            const double* __restrict__ Ax, double* __restrict__ r,
                            const int* __restrict__ tmask) {
    int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (e >= tot) return;
    if (!tmask[rbprob[(e / k) >> 8]]) return;
    if (col_of(st, rbprob, e, k).active) r[e] = b[e] - Ax[e];
}

__global__ void k_btrue_final(const double* __restrict__ prr, const int* __restrict__ rbrange,
                              int P, int k, double tol, BCol* __restrict__ st,
                              BFlags* __restrict__ fl, int* __restrict__ live_prob,
                              int* __restrict__ broke_prob,
                              unsigned long long* __restrict__ maxtru_bits,
                              int* __restrict__ act_prob, const int* __restrict__ tmask) {
    unsigned long long* __restrict__ maxgap_bits = maxtru_bits + P;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= P * k) return;
    const int b = e / k, c = e - b * k;
    BCol s = st[e];
    if (!tmask[b]) {
        // problem not in this replacement: state unchanged, flags as k_brr
        if (s.active) {
            atomicAdd(&fl->live, 1);
            atomicOr(&act_prob[b], 1);
            if (!s.parked) {
                atomicAdd(&fl->pending, 1);
                atomicOr(&live_prob[b], 1);
            }
        }
        if (s.status == PKM_COL_BREAKDOWN) {
            atomicAdd(&fl->broke, 1);
            atomicAdd(&broke_prob[b], 1);
        }
        return;
    }
    double gap = 0.0;
    if (s.active) {
        const double rr = bsum(prr, rbrange, b, k, c);
        s.rr = rr;
        const double rec_before = s.rec;
        s.tru = s.rec = s.bnorm > 0.0 ? sqrt(rr) / s.bnorm : 0.0;
        gap = s.tru / fmax(rec_before, 1e-300);
        if (!isfinite(rr)) {
            s.active = 0;
            s.status = PKM_COL_BREAKDOWN;
        } else if (s.tru <= tol) {
            s.active = 0;
            s.status = PKM_COL_CONVERGED;
        } else {
            s.ref = s.tru;
            if (s.eta > 0.0) s.restart = 1;
        }
        s.parked = 0;
    }
    if (s.active) {
        atomicAdd(&fl->live, 1);
        atomicAdd(&fl->pending, 1);
        atomicOr(&live_prob[b], 1);
        atomicOr(&act_prob[b], 1);
        // non-negative doubles order like their bit patterns
        atomicMax(&maxtru_bits[b], (unsigned long long)__double_as_longlong(s.tru));
        if (isfinite(gap))
            atomicMax(&maxgap_bits[b], (unsigned long long)__double_as_longlong(gap));
    }
    if (s.status == PKM_COL_BREAKDOWN) {
        atomicAdd(&fl->broke, 1);
        atomicAdd(&broke_prob[b], 1);
    }
    st[e] = s;
}

// problems with esc[b] = 1: broken columns resume, active columns restart
// (beta = 0) in plain replacement mode.  esc[b] = 2: active columns restart
// and enter refinement mode with parameter eta.
__global__ void k_breactivate(int P, int k, const int* __restrict__ esc, double eta,
                              BCol* __restrict__ st) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= P * k || !esc[e / k]) return;
    const int mode = esc[e / k];
    BCol s = st[e];
    if (mode == 1 && s.status == PKM_COL_BREAKDOWN) {
        s.active = 1;
        s.status = PKM_COL_CONVERGED;
        s.parked = 0;
    }
    if (s.active) {
        s.restart = 1;
        s.eta = mode == 2 ? eta : 0.0;
        s.ref = s.tru;
    }
    st[e] = s;
}

__global__ void k_bbeta(const double* __restrict__ prz, const int* __restrict__ rbrange, int P,
                        int k, BCol* __restrict__ st) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= P * k) return;
    const int b = e / k, c = e - b * k;
    BCol s = st[e];
    if (bstep(s)) {
        const double rz = bsum(prz, rbrange, b, k, c);
        if (rz < 0.0 || !isfinite(rz)) {
            s.active = 0;
            s.status = PKM_COL_BREAKDOWN;
            s.beta = 0.0;
        } else {
            s.beta = (s.rz > 0.0 && !s.restart) ? rz / s.rz : 0.0;
            s.rz = rz;
            s.restart = 0;
        }
    } else {
        s.beta = 0.0;
    }
    st[e] = s;
}

__global__ void k_bupdate_p(int64_t tot, int k, const int* __restrict__ rbprob,
                            const BCol* __restrict__ st, const double* __restrict__ z,
                            double* __restrict__ p) {
    int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (e >= tot) return;
    const BCol& s = col_of(st, rbprob, e, k);
    if (bstep(s)) p[e] = fma(s.beta, p[e], z[e]);
}

__global__ void k_bmark_maxiter(int P, int k, BCol* __restrict__ st) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < P * k && st[e].active) {
        st[e].active = 0;
        st[e].status = PKM_COL_MAX_ITER;
    }
}

__global__ void k_breport(const double* __restrict__ prr, const int* __restrict__ rbrange, int P,
                          int k, BCol* __restrict__ st, const int* __restrict__ tmask) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= P * k) return;
    const int b = e / k, c = e - b * k;
    if (!tmask[b]) return;   // certified columns keep the residual of their certification
    const double rr = bsum(prr, rbrange, b, k, c);
    st[e].tru = st[e].bnorm > 0.0 ? sqrt(rr) / st[e].bnorm : 0.0;
}

__global__ void k_bsub(int64_t tot, const double* __restrict__ a, const double* __restrict__ b,
                       double* __restrict__ out) {
    int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (e < tot) out[e] = a[e] - b[e];
}

// ---------------------------------------------------------------------------
// batched Woodbury apply: Z = D^-1 R - Psi (Psi^T R) per problem
// ---------------------------------------------------------------------------
typedef double f64x4 __attribute__((ext_vector_type(4)));

// items: (problem, 64-column block of Psi, row chunk)
template <int KT>
__global__ __launch_bounds__(256) void k_bpsit_r(const BDesc* __restrict__ desc,
                                                 const int4* __restrict__ items,
                                                 const int* __restrict__ live,
                                                 const double* __restrict__ R, int k,
                                                 double* __restrict__ part) {
    const int4 item = items[blockIdx.x];
    if (!live[item.x]) return;
    const BDesc D = desc[item.x];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int g = lane >> 4, cc = lane & 15;
    const int j0 = (item.y * 4 + w) * 16;
    if (j0 >= D.m) return;
    const int m = D.m;
    const int64_t i0 = int64_t(item.z) * D.rpc;
    const int64_t i1 = min(D.n, i0 + D.rpc);
    const int jj = j0 + cc;
    const bool jv = jj < m;
    f64x4 acc[KT];
#pragma unroll
    for (int kt = 0; kt < KT; ++kt) acc[kt] = f64x4{0.0, 0.0, 0.0, 0.0};
    for (int64_t ib = i0; ib < i1; ib += 16) {
        double a[4], bb[4][KT];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t i = ib + 4 * g + q;
            const bool iv = i < i1;
            a[q] = (iv && jv) ? D.psi[i * m + jj] : 0.0;
#pragma unroll
            for (int kt = 0; kt < KT; ++kt) {
                const int c = 16 * kt + cc;
                bb[q][kt] = (iv && c < k) ? R[(D.row0 + i) * k + c] : 0.0;
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int kt = 0; kt < KT; ++kt)
                acc[kt] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[q], bb[q][kt], acc[kt], 0, 0, 0);
    }
#pragma unroll
    for (int kt = 0; kt < KT; ++kt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int j = j0 + g + 4 * r;
            const int c = 16 * kt + cc;
            if (j < m && c < k) part[D.partoff + (int64_t(item.z) * m + j) * k + c] = acc[kt][r];
        }
}

// items: (problem, 64-output block of its padded T)
__global__ __launch_bounds__(256) void k_bsum_chunks(const BDesc* __restrict__ desc,
                                                     const int4* __restrict__ items,
                                                     const int* __restrict__ live,
                                                     const double* __restrict__ part, int k,
                                                     int ldt, double* __restrict__ T) {
    __shared__ double sh[4][64];
    const int4 item = items[blockIdx.x];
    const BDesc D = desc[item.x];
    const bool lv = live[item.x] != 0;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t e = int64_t(item.y) * 64 + lane;
    const bool ev = lv && e < int64_t(D.mpad) * ldt;
    const int j = ev ? int(e / ldt) : 0, c = ev ? int(e % ldt) : 0;
    double s = 0.0;
    if (ev && j < D.m && c < k)
        for (int q = w; q < D.nchunk; q += 4) s += part[D.partoff + (int64_t(q) * D.m + j) * k + c];
    sh[w][lane] = s;
    __syncthreads();
    if (w == 0 && ev) T[D.toff + e] = (sh[0][lane] + sh[1][lane]) + (sh[2][lane] + sh[3][lane]);
}

// items: (problem, 64-row block); problems without a preconditioner copy R.
template <int KT>
__global__ __launch_bounds__(256) void k_bapply_z(const BDesc* __restrict__ desc,
                                                  const int4* __restrict__ items,
                                                  const int* __restrict__ live,
                                                  const double* __restrict__ T, int ldt,
                                                  const double* __restrict__ R, int k,
                                                  double* __restrict__ Z) {
    const int4 item = items[blockIdx.x];
    if (!live[item.x]) return;
    const BDesc D = desc[item.x];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int g = lane >> 4, rr = lane & 15;
    const int64_t lrow0 = (int64_t(item.y) * 4 + w) * 16;
    if (lrow0 >= D.n) return;
    if (D.psi == nullptr) {
        for (int q = 0; q < 4; ++q) {
            const int64_t i = lrow0 + g + 4 * q;
            if (i < D.n)
                for (int c = rr; c < k; c += 16) Z[(D.row0 + i) * k + c] = R[(D.row0 + i) * k + c];
        }
        return;
    }
    const int m = D.m;
    const int64_t row = lrow0 + rr;
    const bool rv = row < D.n;
    const double* prow = D.psi + (rv ? row : 0) * m;
    const double* Tb = T + D.toff;
    f64x4 acc[KT];
#pragma unroll
    for (int kt = 0; kt < KT; ++kt) acc[kt] = f64x4{0.0, 0.0, 0.0, 0.0};
    for (int m0 = 0; m0 < m; m0 += 16) {
        double a[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int mm = m0 + 4 * g + q;
            a[q] = (rv && mm < m) ? prow[mm] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double* trow = Tb + int64_t(m0 + 4 * g + q) * ldt + rr;
#pragma unroll
            for (int kt = 0; kt < KT; ++kt)
                acc[kt] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[q], trow[16 * kt], acc[kt], 0, 0, 0);
        }
    }
#pragma unroll
    for (int kt = 0; kt < KT; ++kt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t i = lrow0 + g + 4 * r;
            const int c = 16 * kt + rr;
            if (i < D.n && c < k) {
                const int64_t e = (D.row0 + i) * k + c;
                Z[e] = D.dinv[i] * R[e] - acc[kt][r];
            }
        }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
struct TuneKey {
    int s4, kt, kr;
    int64_t work_bucket;
    bool operator<(const TuneKey& o) const {
        return std::tie(s4, kt, kr, work_bucket) < std::tie(o.s4, o.kt, o.kr, o.work_bucket);
    }
};

// Tuned launch shape of one product class: i-tiles of 16 rows per wave (U;
// a work-group of 4 waves covers 64 U rows) and the work-group count below
// which a problem's row blocks are split over column ranges of K (fill).
struct TuneVal {
    int u, fill;
};

static std::mutex g_tune_mu;            // guards g_tune and g_tune_loaded
static std::map<TuneKey, TuneVal> g_tune;
static bool g_tune_loaded = false;

// A cached entry is used only if its shape is one the launchers instantiate
// for its key: FP16x3 keys (s4 = 100 + BF16 slices 1..7, kt 1..3, kr = merged
// last tile 0/1) take U in {2, 4}; FP32 keys (s4 = augmented slices 1..9,
// kt 0..2, kr 0/1) take U in {1, 2, 4}; fill in {256, ..., 4096}.
static bool tune_valid(const TuneKey& k, const TuneVal& v) {
    const bool f16 = k.s4 >= 100;
    const bool key_ok = f16 ? (k.s4 <= 107 && k.kt >= 1 && k.kt <= 3 && (k.kr == 0 || k.kr == 1))
                            : (k.s4 >= 1 && k.s4 <= 9 && k.kt >= 0 && k.kt <= 2 &&
                               (k.kr == 0 || k.kr == 1) && k.kt + k.kr >= 1);
    const bool u_ok = f16 ? (v.u == 2 || v.u == 4) : (v.u == 1 || v.u == 2 || v.u == 4);
    const bool fill_ok = v.fill == 256 || v.fill == 512 || v.fill == 1024 || v.fill == 2048 ||
                         v.fill == 4096;
    return key_ok && u_ok && fill_ok && k.work_bucket >= 1 &&
           (k.work_bucket & (k.work_bucket - 1)) == 0;
}

// One JSON line of the cache file; entries written before the fill field
// existed take fill 1024 (the earlier fixed value).
static bool tune_parse(const char* line, TuneKey* k, TuneVal* v) {
    long long wb = 0;
    int u = 0, fill = 1024;
    const int got = std::sscanf(line, " {\"s4\": %d, \"kt\": %d, \"kr\": %d, \"work\": %lld, \"u\": %d, \"fill\": %d",
                                &k->s4, &k->kt, &k->kr, &wb, &u, &fill);
    if (got < 5) return false;
    k->work_bucket = wb;
    *v = TuneVal{u, fill};
    return tune_valid(*k, *v);
}

// Merges the valid entries of a cache file into the in-memory cache (caller
// holds g_tune_mu); counts accepted and rejected non-empty lines.
static void tune_merge_file(const char* path, int* accepted, int* rejected) {
    std::ifstream f(path);
    std::string line;
    while (std::getline(f, line)) {
        if (line.find_first_not_of(" \t\r") == std::string::npos) continue;
        TuneKey k{};
        TuneVal v{};
        if (tune_parse(line.c_str(), &k, &v)) {
            g_tune[k] = v;
            ++*accepted;
        } else {
            ++*rejected;
        }
    }
}

static void tune_load() {   // caller holds g_tune_mu
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char* path = std::getenv("PKM_TUNE_CACHE");
    if (!path) return;
    int a = 0, r = 0;
    tune_merge_file(path, &a, &r);
}

static void tune_save() {   // caller holds g_tune_mu
    const char* path = std::getenv("PKM_TUNE_CACHE");
    if (!path) return;
    std::ofstream f(path);
    for (auto& kv : g_tune)
        f << "{\"s4\": " << kv.first.s4 << ", \"kt\": " << kv.first.kt << ", \"kr\": " << kv.first.kr
          << ", \"work\": " << kv.first.work_bucket << ", \"u\": " << kv.second.u
          << ", \"fill\": " << kv.second.fill << "}\n";
}

template <int S4, int KT, int KR>
static void launch_bmvm_u(int U, int grid, hipStream_t s, const BDesc* desc, const int4* items,
                          int nitems, int* counter, const int* live, const int* use64,
                          const float* vs, float* y, int64_t ss) {
    if (U == 4)
        k_bmvm_f32<S4, KT, KR, 4><<<grid, 256, 0, s>>>(desc, items, nitems, counter, live, use64, vs, y, ss);
    else if (U == 2)
        k_bmvm_f32<S4, KT, KR, 2><<<grid, 256, 0, s>>>(desc, items, nitems, counter, live, use64, vs, y, ss);
    else
        k_bmvm_f32<S4, KT, KR, 1><<<grid, 256, 0, s>>>(desc, items, nitems, counter, live, use64, vs, y, ss);
}

template <int S4>
static void launch_bmvm_s(int KT, int KR, int U, int grid, hipStream_t s, const BDesc* desc,
                          const int4* items, int nitems, int* counter, const int* live,
                          const int* use64, const float* vs, float* y, int64_t ss) {
#define PKM_BB(kt, kr)                                                                             \
    if (KT == kt && KR == kr) {                                                                    \
        launch_bmvm_u<S4, kt, kr>(U, grid, s, desc, items, nitems, counter, live, use64, vs, y, ss); \
        return;                                                                                    \
    }
    PKM_BB(0, 1) PKM_BB(1, 0) PKM_BB(1, 1) PKM_BB(2, 0) PKM_BB(2, 1)
#undef PKM_BB
    fail(PKM_ERR_UNSUPPORTED, "batched product: k must be <= 33");
}

static void launch_bmvm(int S4, int KT, int KR, int U, int grid, hipStream_t s, const BDesc* desc,
                        const int4* items, int nitems, int* counter, const int* live,
                        const int* use64, const float* vs, float* y, int64_t ss) {
    switch (S4) {
        case 1: launch_bmvm_s<1>(KT, KR, U, grid, s, desc, items, nitems, counter, live, use64, vs, y, ss); break;
        case 2: launch_bmvm_s<2>(KT, KR, U, grid, s, desc, items, nitems, counter, live, use64, vs, y, ss); break;
        case 3: launch_bmvm_s<3>(KT, KR, U, grid, s, desc, items, nitems, counter, live, use64, vs, y, ss); break;
        case 4: launch_bmvm_s<4>(KT, KR, U, grid, s, desc, items, nitems, counter, live, use64, vs, y, ss); break;
        case 5: launch_bmvm_s<5>(KT, KR, U, grid, s, desc, items, nitems, counter, live, use64, vs, y, ss); break;
        case 6: launch_bmvm_s<6>(KT, KR, U, grid, s, desc, items, nitems, counter, live, use64, vs, y, ss); break;
        case 7: launch_bmvm_s<7>(KT, KR, U, grid, s, desc, items, nitems, counter, live, use64, vs, y, ss); break;
        case 8: launch_bmvm_s<8>(KT, KR, U, grid, s, desc, items, nitems, counter, live, use64, vs, y, ss); break;
        case 9: launch_bmvm_s<9>(KT, KR, U, grid, s, desc, items, nitems, counter, live, use64, vs, y, ss); break;
        default: fail(PKM_ERR_UNSUPPORTED, "batched product: d must be <= 34");
    }
}

template <int S6, int KT, bool ML>
static void launch_bmvm16_u(int U, int grid, hipStream_t s, const BDesc* desc, const int4* items,
                            int nitems, int* counter, const int* live, const int* use64,
                            const bbf16x8* vb, const unsigned long long* colmax, int k, float* y,
                            int64_t ss) {
    if (U == 4)
        k_bmvm_f16<S6, KT, 4, ML><<<grid, 256, 0, s>>>(desc, items, nitems, counter, live, use64, vb,
                                                        colmax, k, y, ss);
    else
        k_bmvm_f16<S6, KT, 2, ML><<<grid, 256, 0, s>>>(desc, items, nitems, counter, live, use64, vb,
                                                        colmax, k, y, ss);
}

// KT16 = ceil(k / 16) column tiles, the last merged (ML) when it holds <= 8
template <int S6>
static void launch_bmvm16_s(int KT, bool ml, int U, int grid, hipStream_t s, const BDesc* desc,
                            const int4* items, int nitems, int* counter, const int* live,
                            const int* use64, const bbf16x8* vb,
                            const unsigned long long* colmax, int k, float* y, int64_t ss) {
#define PKM_BH(kt, m)                                                                              \
    if (KT == kt && ml == m) {                                                                     \
        launch_bmvm16_u<S6, kt, m>(U, grid, s, desc, items, nitems, counter, live, use64, vb,      \
                                   colmax, k, y, ss);                                              \
        return;                                                                                    \
    }
    PKM_BH(1, true) PKM_BH(1, false) PKM_BH(2, true) PKM_BH(2, false) PKM_BH(3, true)
#undef PKM_BH
    fail(PKM_ERR_UNSUPPORTED, "batched FP16x3 product: k must be <= 33");
}

static void launch_bmvm16(int S6, int KT, bool ml, int U, int grid, hipStream_t s,
                          const BDesc* desc, const int4* items, int nitems, int* counter,
                          const int* live, const int* use64, const bbf16x8* vb,
                          const unsigned long long* colmax, int k, float* y, int64_t ss) {
#define PKM_BS(s6)                                                                                 \
    case s6:                                                                                       \
        launch_bmvm16_s<s6>(KT, ml, U, grid, s, desc, items, nitems, counter, live, use64, vb,     \
                            colmax, k, y, ss);                                                     \
        break;
    switch (S6) {
        PKM_BS(1) PKM_BS(2) PKM_BS(3) PKM_BS(4) PKM_BS(5) PKM_BS(6) PKM_BS(7)
        default: fail(PKM_ERR_UNSUPPORTED, "batched FP16x3 product: d must be <= 36");
    }
#undef PKM_BS
}

struct ClassPlan {
    int s4;
    std::vector<int> probs;
    int U = 4;
    int64_t work = 0;           // sum of n_pad^2 / 256
    DevBuf items;               // int4 (problem, row block, split, splits)
    int nitems = 0;
};

int solve_batched(pkm_ctx* ctx, int P, const pkm_problem* probs, const pkm_precond* const* pcs,
                  int k, const double* const* B, double* const* X, const pkm_solve_opts* o,
                  pkm_solve_info* infos) {
    hipStream_t s = ctx->stream;
    auto t_start = std::chrono::steady_clock::now();
    const int prec = o->prec;
    PKM_REQUIRE(prec == PKM_FP32 || prec == PKM_FP64 || prec == PKM_F16X3,
                "batched solve supports FP32, F16X3 or FP64 products");
    PKM_REQUIRE(k >= 1 && k <= 33, "batched solve supports 1 <= k <= 33");
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        tune_load();
    }

    // per-problem prepared operands and packed layout (released on every exit)
    struct Preps {
        pkm_ctx* ctx;
        std::vector<Prepared> v;
        ~Preps() {
            ctx->active = &ctx->prep;
            for (auto& q : v) {
                q.xs64.release();
                q.jside64.release();
                q.iside64.release();
                q.jside.release();
                q.iside.release();
                q.jsb.release();
                q.isb.release();
            }
        }
    } holder{ctx, std::vector<Prepared>(P)};
    std::vector<Prepared>& preps = holder.v;
    std::vector<BDesc> hd(P);
    std::vector<int64_t> row0(P + 1, 0);
    for (int b = 0; b < P; ++b) {
        ctx->active = &preps[b];
        prepare(ctx, &probs[b], true, prec != PKM_FP64);
        if (prec == PKM_F16X3) prepare_bf16(ctx);
        ctx->active = &ctx->prep;
        row0[b + 1] = row0[b] + round_up(probs[b].n, 256);
    }
    const int64_t ntot = row0[P];
    const int nrb = int(ntot / 256);
    std::vector<int> rbprob(nrb), rbrange(P + 1);
    for (int b = 0; b < P; ++b) {
        rbrange[b] = int(row0[b] / 256);
        for (int64_t rb = row0[b] / 256; rb < row0[b + 1] / 256; ++rb) rbprob[rb] = b;
    }
    rbrange[P] = nrb;
    // preconditioner partial-sum layout
    int KT = k / 16, KR = k % 16;
    if (KR > 1) {
        KT += 1;
        KR = 0;
    }
    const int KP = 16 * KT + KR;
    const int KTa = int(cdiv(k, 16));   // apply column tiles
    const int ldt = 16 * KTa;
    int64_t partoff = 0, toff = 0;
    std::vector<int4> it1, itS, it2;
    for (int b = 0; b < P; ++b) {
        BDesc& D = hd[b];
        D.row0 = row0[b];
        D.n = probs[b].n;
        D.tile0 = row0[b] / 16;
        D.ntiles = preps[b].n_pad / 16;
        D.jside = preps[b].jside.as<float>();
        D.iside = preps[b].iside.as<float>();
        D.jsb = preps[b].jsb.p;
        D.isb = preps[b].isb.p;
        D.sigma2 = probs[b].sigma2;
        D.lambda = probs[b].lambda;
        const pkm_precond* pc = pcs ? pcs[b] : nullptr;
        D.psi = pc ? pc->psi.as<double>() : nullptr;
        D.dinv = pc ? pc->dinv.as<double>() : nullptr;
        D.m = pc ? pc->m : 0;
        if (pc) {
            PKM_REQUIRE(pc->n == probs[b].n, "batched: preconditioner built for another n");
            const int mt = int(cdiv(D.m, 64));
            int64_t nchunk = std::max<int64_t>(1, std::min<int64_t>(cdiv(D.n, 256), 64));
            D.rpc = round_up(cdiv(D.n, nchunk), 16);
            D.nchunk = int(cdiv(D.n, D.rpc));
            D.mpad = int(round_up(D.m, 16));
            D.partoff = partoff;
            D.toff = toff;
            partoff += int64_t(D.nchunk) * D.m * k;
            toff += int64_t(D.mpad) * ldt;
            for (int y = 0; y < mt; ++y)
                for (int z = 0; z < D.nchunk; ++z) it1.push_back({b, y, z, 0});
            for (int y = 0; y < int(cdiv(int64_t(D.mpad) * ldt, 64)); ++y) itS.push_back({b, y, 0, 0});
        }
        for (int y = 0; y < int(cdiv(D.n, 64)); ++y) it2.push_back({b, y, 0, 0});
    }
    // product work lists per dimension class (FP32: augmented 4-slices,
    // FP16x3: BF16 32-slot slices), longest items first
    const bool f16 = prec == PKM_F16X3;
    const int KT16 = int(cdiv(k, 16));
    const bool ml16 = k - 16 * (KT16 - 1) <= 8;   // FP16x3: merged last column tile
    std::map<int, ClassPlan> classes;
    if (prec != PKM_FP64)
        for (int b = 0; b < P; ++b) {
            const int sl = f16 ? preps[b].s6 : preps[b].d4 / 4;
            ClassPlan& cp = classes[sl];
            cp.s4 = sl;
            cp.probs.push_back(b);
            cp.work += preps[b].n_pad * preps[b].n_pad / 256;
        }

    // device buffers (batch workspace)
    auto& W = ctx->batch;
    W[0].ensure(sizeof(BDesc) * P);
    W[1].ensure(sizeof(int) * (nrb + 2 * P + 1));
    const size_t vec = sizeof(double) * ntot * k;
    for (int i = 2; i < 8; ++i) W[i].ensure(vec);   // b, x, r, z, p, Ap
    W[8].ensure(vec);                                  // tmp
    W[9].ensure(sizeof(double) * int64_t(nrb) * k * 2);
    W[10].ensure(sizeof(BCol) * P * k + sizeof(BFlags) + 64);
    W[11].ensure(sizeof(int) * (6 * P + 64) + sizeof(unsigned long long) * 2 * P);   // per-problem flags
    W[12].ensure(sizeof(int4) * (it1.size() + itS.size() + it2.size() + 3));
    W[13].ensure(sizeof(double) * std::max<int64_t>(partoff + toff, 1));
    W[14].ensure(sizeof(float) * (ntot / 16) * 16 * KP + 64);
    constexpr int kMaxSplit = 8;
    const int64_t split_stride = ntot * KP;
    W[15].ensure(sizeof(float) * split_stride * kMaxSplit + 64);
    if (f16) {   // FP16 parts of p (ntot / 32 chunks x KT16 x 2 x 512) and column maxima
        W[16].ensure(sizeof(__bf16) * (ntot / 32) * KT16 * 2 * 512);
        W[17].ensure(sizeof(unsigned long long) * P * k + 64);
        PKM_HIP(hipMemsetAsync(W[16].p, 0, sizeof(__bf16) * (ntot / 32) * KT16 * 2 * 512, s));
        PKM_HIP(hipMemsetAsync(W[17].p, 0, sizeof(unsigned long long) * P * k, s));
    }
    const bbf16x8* vb16 = f16 ? W[16].as<bbf16x8>() : nullptr;
    unsigned long long* colmax16 = f16 ? W[17].as<unsigned long long>() : nullptr;
    BDesc* d_desc = W[0].as<BDesc>();
    int* d_rbprob = W[1].as<int>();
    int* d_rbrange = d_rbprob + nrb;
    int* d_nsplit = d_rbrange + P + 1;   // column-range splits per problem
    double* bb = W[2].as<double>();
    double* x = W[3].as<double>();
    double* r = W[4].as<double>();
    double* z = W[5].as<double>();
    double* p = W[6].as<double>();
    double* Ap = W[7].as<double>();
    double* tmp = W[8].as<double>();
    double* partA = W[9].as<double>();
    double* partB = partA + int64_t(nrb) * k;
    BCol* st = W[10].as<BCol>();
    BFlags* fl = reinterpret_cast<BFlags*>(st + P * k);
    int* live = W[11].as<int>();
    int* counter = live + P;              // 16 ints reserved
    int* use64d = counter + 16;           // P: problem runs on FP64 products
    int* esc = use64d + P;                // P: problem escalates now
    int* brokep = esc + P;                // P: broken columns per problem
    int* actp = brokep + P;               // P: problem has active (maybe parked) columns
    int* tmask = actp + P;                // P: problems in the current FP64 replacement
    unsigned long long* maxtru = reinterpret_cast<unsigned long long*>(
        W[11].as<char>() + round_up(sizeof(int) * (6 * P + 64), 8));
    int4* d_it1 = W[12].as<int4>();
    int4* d_itS = d_it1 + it1.size();
    int4* d_it2 = d_itS + itS.size();
    double* part = W[13].as<double>();
    double* Tpad = part + partoff;
    float* vs = W[14].as<float>();
    float* y32 = W[15].as<float>();
    PKM_HIP(hipMemcpyAsync(d_desc, hd.data(), sizeof(BDesc) * P, hipMemcpyHostToDevice, s));
    PKM_HIP(hipMemcpyAsync(d_rbprob, rbprob.data(), sizeof(int) * nrb, hipMemcpyHostToDevice, s));
    PKM_HIP(hipMemcpyAsync(d_rbrange, rbrange.data(), sizeof(int) * (P + 1), hipMemcpyHostToDevice, s));
    if (!it1.empty()) PKM_HIP(hipMemcpyAsync(d_it1, it1.data(), sizeof(int4) * it1.size(), hipMemcpyHostToDevice, s));
    if (!itS.empty()) PKM_HIP(hipMemcpyAsync(d_itS, itS.data(), sizeof(int4) * itS.size(), hipMemcpyHostToDevice, s));
    PKM_HIP(hipMemcpyAsync(d_it2, it2.data(), sizeof(int4) * it2.size(), hipMemcpyHostToDevice, s));
    // pack b, x0 = 0
    for (int i = 2; i < 9; ++i) PKM_HIP(hipMemsetAsync(W[i].p, 0, vec, s));
    for (int b = 0; b < P; ++b)
        PKM_HIP(hipMemcpyAsync(bb + row0[b] * k, B[b], sizeof(double) * probs[b].n * k,
                               hipMemcpyDeviceToDevice, s));
    const int64_t tot = ntot * k;
    const unsigned gb = unsigned(cdiv(tot, 256));
    const unsigned gpk = unsigned(cdiv(int64_t(P) * k, 256));
    // pinned status slots: slot 0 for synchronous polls, 1 and 2 for the
    // lag-one polls of the loop; each holds the flags, then P ints of "has
    // active columns", then P ints of "has stepping columns"
    const size_t slot_bytes = round_up(size_t(64) + sizeof(int) * 2 * size_t(P), 256);
    auto slot_flags = [&](int q) {
        return reinterpret_cast<BFlags*>(static_cast<char*>(ctx->pinned) + q * slot_bytes);
    };
    auto slot_act = [&](int q) {
        return reinterpret_cast<int*>(static_cast<char*>(ctx->pinned) + q * slot_bytes + 64);
    };
    BFlags* hfl = slot_flags(0);
    int* hact = slot_act(0);
    int* hstep = hact + P;

    auto dots = [&](const double* u, const double* v, double* out) {
        k_bdot_part<<<nrb, 256, 0, s>>>(u, v, k, out);
        PKM_CHECK_LAUNCH();
    };
    auto reset_flags = [&]() {
        PKM_HIP(hipMemsetAsync(fl, 0, sizeof(BFlags), s));
        PKM_HIP(hipMemsetAsync(live, 0, sizeof(int) * P, s));
        PKM_HIP(hipMemsetAsync(actp, 0, sizeof(int) * P, s));
    };
    // host copies (as of the last poll) of the per-problem flags: act = has
    // active columns, ready = has active columns and all of them parked
    std::vector<int> act(P, 1), ready(P, 0), stepping(P, 1);
    auto take = [&](int q) {
        const int* ha = slot_act(q);
        for (int b = 0; b < P; ++b) {
            act[b] = ha[b];
            stepping[b] = ha[P + b];
            ready[b] = ha[b] && !ha[P + b];
        }
        return *slot_flags(q);
    };
    auto enqueue_copy = [&](int q) {
        PKM_HIP(hipMemcpyAsync(slot_flags(q), fl, sizeof(BFlags), hipMemcpyDeviceToHost, s));
        PKM_HIP(hipMemcpyAsync(slot_act(q), actp, sizeof(int) * P, hipMemcpyDeviceToHost, s));
        PKM_HIP(hipMemcpyAsync(slot_act(q) + P, live, sizeof(int) * P, hipMemcpyDeviceToHost, s));
    };
    int lag_slot = -1;   // lagged slot whose copy is still unread (-1: none)
    auto poll = [&]() {
        enqueue_copy(0);
        PKM_HIP(hipStreamSynchronize(s));
        lag_slot = -1;   // in-flight copies completed and are superseded
        return take(0);
    };
    // Lag-one poll (as in pkm_solve): this step's status goes to slot 1 or 2
    // and the host reads the previous poll's slot, so the stream does not
    // drain between steps.  What the loop acts on -- no live column, a
    // problem whose active columns are all parked, a breakdown -- holds until
    // the host itself acts on it, so a late read costs at most one idle step.
    auto poll_lagged = [&](BFlags& out) {
        const int q = lag_slot == 1 ? 2 : 1;
        enqueue_copy(q);
        PKM_HIP(hipEventRecord(ctx->poll_ev[q - 1], s));
        const int prev = lag_slot;
        lag_slot = q;
        if (prev < 0) return false;
        PKM_HIP(hipEventSynchronize(ctx->poll_ev[prev - 1]));
        out = take(prev);
        return true;
    };
    auto apply = [&](const double* R, double* Zo) {
        if (!it1.empty()) {
            switch (KTa) {
                case 1: k_bpsit_r<1><<<unsigned(it1.size()), 256, 0, s>>>(d_desc, d_it1, live, R, k, part); break;
                case 2: k_bpsit_r<2><<<unsigned(it1.size()), 256, 0, s>>>(d_desc, d_it1, live, R, k, part); break;
                default: k_bpsit_r<3><<<unsigned(it1.size()), 256, 0, s>>>(d_desc, d_it1, live, R, k, part); break;
            }
            PKM_CHECK_LAUNCH();
            k_bsum_chunks<<<unsigned(itS.size()), 256, 0, s>>>(d_desc, d_itS, live, part, k, ldt, Tpad);
            PKM_CHECK_LAUNCH();
        }
        switch (KTa) {
            case 1: k_bapply_z<1><<<unsigned(it2.size()), 256, 0, s>>>(d_desc, d_it2, live, Tpad, ldt, R, k, Zo); break;
            case 2: k_bapply_z<2><<<unsigned(it2.size()), 256, 0, s>>>(d_desc, d_it2, live, Tpad, ldt, R, k, Zo); break;
            default: k_bapply_z<3><<<unsigned(it2.size()), 256, 0, s>>>(d_desc, d_it2, live, Tpad, ldt, R, k, Zo); break;
        }
        PKM_CHECK_LAUNCH();
    };
    // Y = K_y V in FP64 for the problems with mask[b] != 0
    auto product64 = [&](const double* V, double* Y, const std::vector<int>& mask) {
        for (int b = 0; b < P; ++b) {
            if (!mask[b]) continue;
            ctx->active = &preps[b];
            mvm(ctx, PKM_FP64, k, V + row0[b] * k, Y + row0[b] * k);
            ctx->active = &ctx->prep;
        }
    };
    const int grid_q = 256 * 8;   // work-queue work-groups (exit when the list is exhausted)
    std::vector<int> hsplit(P, 1);
    std::vector<int> use64(P, prec == PKM_FP64 ? 1 : 0);
    PKM_HIP(hipMemcpyAsync(use64d, use64.data(), sizeof(int) * P, hipMemcpyHostToDevice, s));
    PKM_HIP(hipMemsetAsync(brokep, 0, sizeof(int) * P, s));
    // build the product item lists, tuned per class
    for (auto& kv : classes) {
        ClassPlan& cp = kv.second;
        int64_t wb = 1;
        while (wb < cp.work) wb <<= 1;
        // FP16x3 classes are keyed 100 + slices, (KT16, merged last tile)
        TuneKey key = f16 ? TuneKey{100 + cp.s4, KT16, ml16 ? 1 : 0, wb} : TuneKey{cp.s4, KT, KR, wb};
        // items for U i-tiles per wave; a problem whose row blocks alone give
        // fewer than `fill` work-groups is split over up to kMaxSplit column
        // ranges of at least 16 tiles each
        auto build = [&](int U, int fill) {
            std::vector<std::pair<int64_t, int4>> v;
            for (int b : cp.probs) {
                const int64_t rows_wg = 64 * U;
                const int nblk = int(cdiv(preps[b].n_pad, rows_wg));
                const int64_t ntiles = preps[b].n_pad / 16;
                int ns = 1;
                while (ns < kMaxSplit && int64_t(nblk) * ns < fill && ntiles / (2 * ns) >= 16) ns *= 2;
                hsplit[b] = ns;
                for (int y = 0; y < nblk; ++y)
                    for (int q = 0; q < ns; ++q) v.push_back({preps[b].n_pad, int4{b, y, q, ns}});
            }
            std::stable_sort(v.begin(), v.end(), [](auto& a, auto& c) { return a.first > c.first; });
            std::vector<int4> items(v.size());
            for (size_t i = 0; i < v.size(); ++i) items[i] = v[i].second;
            return items;
        };
        auto run = [&](int U, const std::vector<int4>& items) {
            cp.items.ensure(sizeof(int4) * items.size());
            PKM_HIP(hipMemcpyAsync(cp.items.p, items.data(), sizeof(int4) * items.size(), hipMemcpyHostToDevice, s));
            PKM_HIP(hipMemsetAsync(counter, 0, sizeof(int), s));
            if (f16)
                launch_bmvm16(cp.s4, KT16, ml16, U, grid_q, s, d_desc, cp.items.as<int4>(),
                              int(items.size()), counter, live, use64d, vb16, colmax16, k, y32,
                              split_stride);
            else
                launch_bmvm(cp.s4, KT, KR, U, grid_q, s, d_desc, cp.items.as<int4>(), int(items.size()),
                            counter, live, use64d, vs, y32, split_stride);
            PKM_CHECK_LAUNCH();
            PKM_HIP(hipStreamSynchronize(s));   // items is pageable host memory
        };
        TuneVal tv{};
        bool cached;
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            auto found = g_tune.find(key);
            cached = found != g_tune.end();
            if (cached) tv = found->second;
        }
        if (!cached) {
            // time every (U, fill) once on this batch (all problems live, p = 0)
            std::vector<int> ones(P, 1);
            PKM_HIP(hipMemcpyAsync(live, ones.data(), sizeof(int) * P, hipMemcpyHostToDevice, s));
            float best_ms = 1e30f;
            tv = TuneVal{4, 1024};
            for (int U : {1, 2, 4}) {
                if (f16 && U == 1) continue;   // FP16x3 kernels: 2 or 4 i-tiles per wave
                for (int fill : {512, 1024, 2048}) {
                    auto items = build(U, fill);
                    run(U, items);   // warm
                    PKM_HIP(hipEventRecord(ctx->ev0, s));
                    run(U, items);
                    PKM_HIP(hipEventRecord(ctx->ev1, s));
                    PKM_HIP(hipEventSynchronize(ctx->ev1));
                    float ms = 0.f;
                    PKM_HIP(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
                    if (ms < best_ms) {
                        best_ms = ms;
                        tv = TuneVal{U, fill};
                    }
                }
            }
            std::lock_guard<std::mutex> lk(g_tune_mu);
            g_tune[key] = tv;
            tune_save();
        }
        PKM_REQUIRE(tune_valid(key, tv), "internal: tuned launch shape not instantiated");
        cp.U = tv.u;
        auto items = build(cp.U, tv.fill);
        cp.nitems = int(items.size());
        cp.items.ensure(sizeof(int4) * items.size());
        PKM_HIP(hipMemcpyAsync(cp.items.p, items.data(), sizeof(int4) * items.size(), hipMemcpyHostToDevice, s));
        PKM_HIP(hipStreamSynchronize(s));
    }
    PKM_HIP(hipMemcpyAsync(d_nsplit, hsplit.data(), sizeof(int) * P, hipMemcpyHostToDevice, s));
    auto product = [&](const double* V, double* Y) {
        if (prec == PKM_FP64) {
            product64(V, Y, stepping);
            return;
        }
        if (f16) {
            PKM_HIP(hipMemsetAsync(colmax16, 0, sizeof(unsigned long long) * P * k, s));
            k_bcolmax<<<nrb, 256, 0, s>>>(V, k, d_rbprob, colmax16);
            PKM_CHECK_LAUNCH();
            const int64_t nch = ntot / 32;
            k_bpack_v16<<<cdiv(nch * KT16 * 512, 256), 256, 0, s>>>(
                V, nch, k, KT16, ml16 ? 1 : 0, d_rbprob, d_desc, colmax16, W[16].as<__bf16>());
            PKM_CHECK_LAUNCH();
        } else {
            k_bpack_v32<<<cdiv((ntot / 16) * 16 * KP, 256), 256, 0, s>>>(V, ntot, k, KT, KR, vs);
            PKM_CHECK_LAUNCH();
        }
        const hipEvent_t t0 = ctx->timing ? timing_start(ctx) : nullptr;
        for (auto& kv : classes) {
            ClassPlan& cp = kv.second;
            PKM_HIP(hipMemsetAsync(counter, 0, sizeof(int), s));
            if (f16)
                launch_bmvm16(cp.s4, KT16, ml16, cp.U, grid_q, s, d_desc, cp.items.as<int4>(),
                              cp.nitems, counter, live, use64d, vb16, colmax16, k, y32, split_stride);
            else
                launch_bmvm(cp.s4, KT, KR, cp.U, grid_q, s, d_desc, cp.items.as<int4>(), cp.nitems,
                            counter, live, use64d, vs, y32, split_stride);
            PKM_CHECK_LAUNCH();
        }
        if (t0) {
            // work of the problems the launch processed, as of the host's last
            // status read (which lags the device by at most one step)
            double pairs = 0.0, flops = 0.0;
            for (int b = 0; b < P; ++b) {
                if (!stepping[b] || use64[b]) continue;
                const double pr = double(probs[b].n) * double(probs[b].n);
                pairs += pr;
                flops += pr * (2.0 * probs[b].d + 2.0 * k);
            }
            timing_stop(ctx, t0, prec, pairs, flops);
        }
        k_bfinish32<<<gb, 256, 0, s>>>(y32, split_stride, f16 ? k : KP, ntot, k, d_rbprob, d_desc,
                                       d_nsplit, V, Y);
        PKM_CHECK_LAUNCH();
        for (int b = 0; b < P; ++b)   // escalated problems: FP64 products
            if (use64[b] && stepping[b]) {
                ctx->active = &preps[b];
                mvm(ctx, PKM_FP64, k, V + row0[b] * k, Y + row0[b] * k);
                ctx->active = &ctx->prep;
            }
    };
    int64_t true_count = 0;
    // FP64 residual replacement for the problems in mask
    auto true_residual = [&](const std::vector<int>& mask) {
        PKM_HIP(hipMemcpyAsync(tmask, mask.data(), sizeof(int) * P, hipMemcpyHostToDevice, s));
        product64(x, tmp, mask);
        k_btrue_res<<<gb, 256, 0, s>>>(tot, k, d_rbprob, st, bb, tmp, r, tmask);
        PKM_CHECK_LAUNCH();
        dots(r, r, partA);
        reset_flags();
        PKM_HIP(hipMemsetAsync(maxtru, 0, sizeof(unsigned long long) * 2 * P, s));
        PKM_HIP(hipMemsetAsync(brokep, 0, sizeof(int) * P, s));
        k_btrue_final<<<gpk, 256, 0, s>>>(partA, d_rbrange, P, k, o->tol, st, fl, live, brokep,
                                          maxtru, actp, tmask);
        PKM_CHECK_LAUNCH();
        ++true_count;
    };
    // Per-problem response to a stalled or broken FP32 refinement: a problem
    // whose largest true residual stalls (StallMonitor) first enters
    // refinement mode (restart at every replacement, inner target
    // kRefineEta); stalling again there, or a broken column, moves it to FP64
    // products: its broken columns resume and all its columns restart from
    // the FP64 true residual.  Returns whether some problem moved to FP64;
    // h_escm then marks those problems (they need a fresh true residual).
    std::vector<StallMonitor> mon(P);
    std::vector<unsigned long long> h_maxtru(2 * P);   // largest true residual, largest gap
    std::vector<int> h_broke(P), h_esc(P), h_escm(P), refining(P, 0), refined(P, 0);
    int64_t it = 0;   // PCG steps so far
    auto escalate_check = [&](bool after_true) -> bool {
        if (prec == PKM_FP64) return false;
        PKM_HIP(hipMemcpyAsync(h_broke.data(), brokep, sizeof(int) * P, hipMemcpyDeviceToHost, s));
        if (after_true)
            PKM_HIP(hipMemcpyAsync(h_maxtru.data(), maxtru, sizeof(unsigned long long) * 2 * P,
                                   hipMemcpyDeviceToHost, s));
        PKM_HIP(hipStreamSynchronize(s));
        bool any = false, moved = false;
        for (int b = 0; b < P; ++b) {
            h_esc[b] = 0;
            h_escm[b] = 0;
            if (use64[b]) continue;
            bool stalled = false;
            double mt = 0.0, mg = 0.0;
            if (after_true) {
                std::memcpy(&mt, &h_maxtru[b], sizeof(double));
                std::memcpy(&mg, &h_maxtru[P + b], sizeof(double));
                stalled = mon[b].stalled(mt, it);
            }
            // diverging (true residual above the right-hand side while the
            // recursion believes it 100 times smaller), broken, or stalled
            // again in refinement mode: FP64 products
            const bool diverging = mt > 1.0 && mg > 100.0;
            if (h_broke[b] > 0 || diverging || (stalled && refining[b])) {
                h_esc[b] = 1;
                h_escm[b] = 1;
                use64[b] = 1;
                refining[b] = 0;
                mon[b].reset();
                any = moved = true;
            } else if (stalled) {
                h_esc[b] = 2;
                refining[b] = 1;
                refined[b] = 1;
                mon[b].reset();
                any = true;
            }
        }
        if (!any) return false;
        PKM_HIP(hipMemcpyAsync(esc, h_esc.data(), sizeof(int) * P, hipMemcpyHostToDevice, s));
        PKM_HIP(hipMemcpyAsync(use64d, use64.data(), sizeof(int) * P, hipMemcpyHostToDevice, s));
        k_breactivate<<<gpk, 256, 0, s>>>(P, k, esc, kRefineEta, st);
        PKM_CHECK_LAUNCH();
        return moved;
    };

    // r0 = b, z0 = P^-1 r0, p0 = z0
    PKM_HIP(hipMemcpyAsync(r, bb, vec, hipMemcpyDeviceToDevice, s));
    {
        std::vector<int> ones(P, 1);
        PKM_HIP(hipMemcpyAsync(live, ones.data(), sizeof(int) * P, hipMemcpyHostToDevice, s));
    }
    apply(r, z);
    PKM_HIP(hipMemcpyAsync(p, z, vec, hipMemcpyDeviceToDevice, s));
    dots(bb, bb, partA);
    dots(r, z, partB);
    k_binit<<<gpk, 256, 0, s>>>(partA, partB, d_rbrange, P, k, st);
    PKM_CHECK_LAUNCH();
    dots(r, r, partA);
    reset_flags();
    k_brr<<<gpk, 256, 0, s>>>(partA, d_rbrange, P, k, o->tol, st, fl, live, brokep, actp);
    PKM_CHECK_LAUNCH();
    BFlags f = poll();
    // FP64 replacement for the problems in mask, then the escalation test
    // PKM_VERBOSE=1 reports every replacement round on stderr (long solves)
    // read per call: a caller may switch progress reports on for one long solve
    const bool verbose = std::getenv("PKM_VERBOSE") != nullptr;
    auto replace = [&](const std::vector<int>& mask) {
        true_residual(mask);
        f = poll();
        if (escalate_check(true)) {
            true_residual(h_escm);
            f = poll();
        }
        if (verbose) {
            int n64 = 0, nref = 0, nact = 0;
            for (int b = 0; b < P; ++b) {
                n64 += use64[b];
                nref += refining[b];
                nact += act[b];
            }
            std::fprintf(stderr, "pkm_solve_batched: step %lld, %d of %d problems live, "
                         "%d in refinement mode, %d on FP64 products, %d live columns\n",
                         (long long)it, nact, P, nref, n64, f.live);
        }
    };
    auto any_of = [](const std::vector<int>& v) {
        return std::any_of(v.begin(), v.end(), [](int q) { return q != 0; });
    };
    if (f.live > 0 && any_of(ready)) replace(ready);
    while (f.live > 0 && it < o->max_iter) {
        product(p, Ap);
        dots(p, Ap, partA);
        k_balpha<<<gpk, 256, 0, s>>>(partA, d_rbrange, P, k, st, fl, live, brokep, actp);
        PKM_CHECK_LAUNCH();
        k_bupdate_xr<<<gb, 256, 0, s>>>(tot, k, d_rbprob, st, p, Ap, x, r);
        PKM_CHECK_LAUNCH();
        dots(r, r, partA);
        k_brr<<<gpk, 256, 0, s>>>(partA, d_rbrange, P, k, o->tol, st, fl, live, brokep, actp);
        PKM_CHECK_LAUNCH();
        ++it;
        // (a negative period is taken as its magnitude, fixed)
        const int every = o->reliable_every < 0 ? -o->reliable_every : o->reliable_every;
        bool do_true = prec != PKM_FP64 && it % every == 0;
        bool have = false;
        if (!do_true && (it % o->check_every == 0 || it == o->max_iter)) {
            if (it == o->max_iter) {
                f = poll();
                have = true;
            } else {
                have = poll_lagged(f);
            }
        }
        if (have) {
            if (f.broke > 0 && escalate_check(false)) {
                true_residual(h_escm);   // reactivated columns get their FP64 residual
                f = poll();
            }
            if (f.live == 0) break;
            // problems whose active columns have all reached the tolerance on
            // the recursive residual are certified (or resume) right away
            if (!do_true && any_of(ready)) {
                replace(ready);
                if (f.live == 0) break;
            }
        }
        if (do_true) {
            replace(act);
            if (f.live == 0) break;
        }
        if (it == o->max_iter) break;
        apply(r, z);
        dots(r, z, partB);
        k_bbeta<<<gpk, 256, 0, s>>>(partB, d_rbrange, P, k, st);
        PKM_CHECK_LAUNCH();
        k_bupdate_p<<<gb, 256, 0, s>>>(tot, k, d_rbprob, st, z, p);
        PKM_CHECK_LAUNCH();
    }
    k_bmark_maxiter<<<gpk, 256, 0, s>>>(P, k, st);
    PKM_CHECK_LAUNCH();
    // final FP64 residual for problems with a column that was not certified
    {
        std::vector<BCol> hs0(size_t(P) * k);
        PKM_HIP(hipMemcpyAsync(hs0.data(), st, sizeof(BCol) * P * k, hipMemcpyDeviceToHost, s));
        PKM_HIP(hipStreamSynchronize(s));
        std::vector<int> need(P, 0);
        for (int b = 0; b < P; ++b)
            for (int c = 0; c < k; ++c)
                if (hs0[size_t(b) * k + c].status != PKM_COL_CONVERGED) need[b] = 1;
        if (any_of(need)) {
            PKM_HIP(hipMemcpyAsync(tmask, need.data(), sizeof(int) * P, hipMemcpyHostToDevice, s));
            product64(x, tmp, need);
            k_bsub<<<gb, 256, 0, s>>>(tot, bb, tmp, tmp);
            PKM_CHECK_LAUNCH();
            dots(tmp, tmp, partA);
            k_breport<<<gpk, 256, 0, s>>>(partA, d_rbrange, P, k, st, tmask);
            PKM_CHECK_LAUNCH();
            PKM_HIP(hipStreamSynchronize(s));   // need is pageable host memory
        }
    }
    for (int b = 0; b < P; ++b)
        PKM_HIP(hipMemcpyAsync(X[b], x + row0[b] * k, sizeof(double) * probs[b].n * k,
                               hipMemcpyDeviceToDevice, s));
    std::vector<BCol> hs(size_t(P) * k);
    PKM_HIP(hipMemcpyAsync(hs.data(), st, sizeof(BCol) * P * k, hipMemcpyDeviceToHost, s));
    PKM_HIP(hipStreamSynchronize(s));
    auto t_end = std::chrono::steady_clock::now();
    int code = PKM_OK;
    for (int b = 0; b < P; ++b)
        for (int c = 0; c < k; ++c) {
            const BCol& h = hs[size_t(b) * k + c];
            if (h.status == PKM_COL_BREAKDOWN) code = PKM_ERR_BREAKDOWN;
            else if (h.status == PKM_COL_MAX_ITER && code == PKM_OK) code = PKM_NOT_CONVERGED;
            if (infos) {
                pkm_solve_info& inf = infos[b];
                if (inf.iters) inf.iters[c] = h.iters;
                if (inf.relres_true) inf.relres_true[c] = h.tru;
                if (inf.relres_rec) inf.relres_rec[c] = h.rec;
                if (inf.col_status) inf.col_status[c] = h.status;
            }
        }
    if (infos)
        for (int b = 0; b < P; ++b) {
            infos[b].prec_final = use64[b] ? PKM_FP64 : prec;
            infos[b].refined = refined[b];
            infos[b].total_iters = it;
            infos[b].true_residuals = true_count;
            infos[b].solve_ms = std::chrono::duration<double, std::milli>(t_end - t_start).count();
        }
    if (code == PKM_ERR_BREAKDOWN) ctx->err = "batched solve: a column broke down";
    else if (code == PKM_NOT_CONVERGED) ctx->err = "batched solve: a column reached max_iter";
    return code;
}

void tune_cache_load(const char* path, int* accepted, int* rejected) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_load();   // the PKM_TUNE_CACHE file first, so that this file's entries win
    tune_merge_file(path, accepted, rejected);
}

}  // namespace pkm
