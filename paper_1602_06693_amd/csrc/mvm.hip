// Matrix-free kernel products Y = (K + lambda I) V (Section 2.1: the O(n^2)
// operation of every CG step).  K is never stored; every tile of Eq. (1) is
// regenerated from the prepared inputs.
//
// FP32 path (one fused kernel per product):
//   for a wave's 16-row i-tiles and each 16-row j-tile
//     S^T = B_j A_i^T            16x16x4 FP32 MFMA over the augmented slots,
//                                giving the base-2 exponent of k(x_i, x_j)
//     K   = exp2(S)              v_exp_f32, in registers
//     Y_i += K V_j               16x16x4 FP32 MFMA per 16 RHS columns, plus
//                                VALU FMAs for a remainder of 1..3 columns
//   Computing the transposed exponent tile leaves, in every lane, four
//   kernel entries of one row i at four consecutive j -- exactly the A
//   operand layout of the K V MFMA, so no LDS round trip is needed.
//   V is packed once per product into MFMA lane order, so every lane's
//   operands are one contiguous 16-byte load.
//   Grid: row blocks x j-splits.  Work-group b runs on XCD b % 8; all
//   work-groups of one XCD take the same j-split so that split's operand
//   stream stays resident in that XCD's L2.
//   The lambda V term is added in FP64 by the consumer of the partial sums.
//
// FP64 path: direct coordinate differences, FP64 exp and FMA on the vector
// ALUs, j-tiles staged in LDS; used for FP64 solves and for the FP64 true
// residual of the reliable-update loop.

#include "pkm_internal.h"

#include <algorithm>

namespace pkm {

typedef float f32x4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// FP32 fused kernel
// ---------------------------------------------------------------------------
template <int S4, int KT, int KR, int U>
__global__ __launch_bounds__(256) void k_mvm_f32(
    const float* __restrict__ jside, const float* __restrict__ iside,
    const float* __restrict__ vs, float* __restrict__ yout, int ntiles, int nrb,
    int jsplit, int tiles_per_split, int64_t split_stride) {
    constexpr int KP = 16 * KT + KR;   // floats per packed V row
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int b = blockIdx.x;
    const int xcd = b & 7, slot = b >> 3;
    const int group = 8 / jsplit;
    const int split = xcd % jsplit;
    const int rb = slot * group + xcd / jsplit;
    if (rb >= nrb) return;
    const int itile0 = (rb * 4 + wave) * U;

    float bi[U][S4];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
        for (int s = 0; s < S4; ++s) bi[u][s] = iside[(int64_t(itile0 + u) * 64 + lane) * S4 + s];

    f32x4 acc[U][KT > 0 ? KT : 1];
    float racc[U][KR > 0 ? KR : 1];
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
        for (int q = 0; q < (KT > 0 ? KT : 1); ++q) acc[u][q] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int e = 0; e < (KR > 0 ? KR : 1); ++e) racc[u][e] = 0.f;
    }

    const int g = lane >> 4;
    const int t0 = split * tiles_per_split;
    const int t1 = min(ntiles, t0 + tiles_per_split);
    for (int t = t0; t < t1; ++t) {
        float aj[S4];
#pragma unroll
        for (int s = 0; s < S4; ++s) aj[s] = jside[(int64_t(t) * 64 + lane) * S4 + s];
        const float* vt = vs + int64_t(t) * 16 * KP;
        f32x4 vv[KT > 0 ? KT : 1];
#pragma unroll
        for (int q = 0; q < KT; ++q) vv[q] = *reinterpret_cast<const f32x4*>(vt + q * 256 + lane * 4);
        f32x4 yr[KR > 0 ? KR : 1];
#pragma unroll
        for (int e = 0; e < KR; ++e)
            yr[e] = *reinterpret_cast<const f32x4*>(vt + KT * 256 + e * 16 + g * 4);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            f32x4 st = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int s = 0; s < S4; ++s)
                st = __builtin_amdgcn_mfma_f32_16x16x4f32(aj[s], bi[u][s], st, 0, 0, 0);
            float kv[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) kv[r] = __builtin_amdgcn_exp2f(st[r]);
#pragma unroll
            for (int q = 0; q < KT; ++q)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    acc[u][q] = __builtin_amdgcn_mfma_f32_16x16x4f32(kv[r], vv[q][r], acc[u][q], 0, 0, 0);
#pragma unroll
            for (int e = 0; e < KR; ++e)
                racc[u][e] += kv[0] * yr[e][0] + kv[1] * yr[e][1] + kv[2] * yr[e][2] + kv[3] * yr[e][3];
        }
    }

    float* yo = yout + int64_t(split) * split_stride;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int64_t row0 = int64_t(itile0 + u) * 16;
#pragma unroll
        for (int q = 0; q < KT; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                yo[(row0 + 4 * g + r) * KP + 16 * q + (lane & 15)] = acc[u][q][r];
#pragma unroll
        for (int e = 0; e < KR; ++e) {
            float v = racc[u][e];
            v += __shfl_xor(v, 16);
            v += __shfl_xor(v, 32);
            if (g == 0) yo[(row0 + (lane & 15)) * KP + 16 * KT + e] = v;
        }
    }
}

// Pack V (n x k FP64, leading dimension ldv) into MFMA lane-order tiles:
//   tile t, column tile q, lane l, r:  V[16 t + 4 (l / 16) + r][16 q + l % 16]
//   remainder column e, row jj:        V[16 t + jj][16 KT + e]
// Rows >= n and columns >= k are zero.
__global__ void k_pack_v32(const double* __restrict__ V, int64_t ldv, int64_t n, int k,
                           int ntiles, int KT, int KR, float* __restrict__ vs) {
    const int KP = 16 * KT + KR;
    int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    int64_t tot = int64_t(ntiles) * 16 * KP;
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
        int ee = w2 >> 4, jj = w2 & 15;
        row = 16 * t + jj;
        col = 16 * KT + ee;
    }
    float v = 0.f;
    if (row < n && col < k) v = float(V[row * ldv + col]);
    vs[e] = v;
}

struct F32Cfg {
    int KT, KR;
};

static F32Cfg f32_cfg(int k) {
    // columns handled by MFMA tiles of 16 and at most one VALU column
    int KT = k / 16, KR = k % 16;
    if (KR > 1) {
        KT += 1;
        KR = 0;
    }
    return {KT, KR};
}

template <int S4>
static void launch_f32_s(F32Cfg c, dim3 grid, hipStream_t s, const float* js,
                         const float* is, const float* vs, float* y, int ntiles, int nrb,
                         int jsplit, int tps, int64_t stride) {
#define PKM_F32_CASE(kt, kr)                                                              \
    if (c.KT == kt && c.KR == kr) {                                                       \
        k_mvm_f32<S4, kt, kr, 4><<<grid, 256, 0, s>>>(js, is, vs, y, ntiles, nrb, jsplit, \
                                                       tps, stride);                      \
        return;                                                                           \
    }
    PKM_F32_CASE(0, 1) PKM_F32_CASE(1, 0) PKM_F32_CASE(1, 1) PKM_F32_CASE(2, 0)
    PKM_F32_CASE(2, 1) PKM_F32_CASE(3, 0) PKM_F32_CASE(3, 1) PKM_F32_CASE(4, 0)
    PKM_F32_CASE(4, 1)
#undef PKM_F32_CASE
    fail(PKM_ERR_UNSUPPORTED, "FP32 product: unsupported column count");
}

F32Out mvm_k32(pkm_ctx* ctx, int k, const double* V, int ldv) {
    Prepared& P = ctx->P();
    PKM_REQUIRE(P.valid32, "internal: FP32 operands not prepared");
    PKM_REQUIRE(k >= 1 && k <= 65, "FP32 product supports 1 <= k <= 65 columns per call");
    F32Cfg c = f32_cfg(k);
    const int KP = 16 * c.KT + c.KR;
    const int ntiles = int(P.n_pad / 16);
    hipStream_t s = ctx->stream;

    ctx->v32.ensure(sizeof(float) * int64_t(ntiles) * 16 * KP);
    int64_t tot = int64_t(ntiles) * 16 * KP;
    k_pack_v32<<<cdiv(tot, 256), 256, 0, s>>>(V, ldv, P.n, k, ntiles, c.KT, c.KR,
                                               ctx->v32.as<float>());
    PKM_CHECK_LAUNCH();

    // launch shape: rows per work-group = 64 U; enough work-groups to fill
    // 256 CUs several times over; j-split divides 8 (XCD mapping)
    constexpr int U = 4;   // i-tiles per wave: 256 rows per work-group
    int64_t nrb = cdiv(P.n_pad, 64 * U);
    int jsplit = 1;
    while (jsplit < 8 && nrb * jsplit < 2048 && ntiles / (jsplit * 2) >= 16) jsplit <<= 1;
    int tps = int(cdiv(ntiles, jsplit));
    int group = 8 / jsplit;
    int64_t nrb_pad = round_up(nrb, group);
    dim3 grid((unsigned)(nrb_pad * jsplit));
    int64_t stride = P.n_pad * KP;
    ctx->y32.ensure(sizeof(float) * stride * jsplit);

    const hipEvent_t t0 = ctx->timing ? timing_start(ctx) : nullptr;
    const float* js = P.jside.as<float>();
    const float* is = P.iside.as<float>();
    float* y = ctx->y32.as<float>();
    switch (P.d4 / 4) {
        case 1: launch_f32_s<1>(c, grid, s, js, is, ctx->v32.as<float>(), y, ntiles, int(nrb), jsplit, tps, stride); break;
        case 2: launch_f32_s<2>(c, grid, s, js, is, ctx->v32.as<float>(), y, ntiles, int(nrb), jsplit, tps, stride); break;
        case 3: launch_f32_s<3>(c, grid, s, js, is, ctx->v32.as<float>(), y, ntiles, int(nrb), jsplit, tps, stride); break;
        case 4: launch_f32_s<4>(c, grid, s, js, is, ctx->v32.as<float>(), y, ntiles, int(nrb), jsplit, tps, stride); break;
        case 5: launch_f32_s<5>(c, grid, s, js, is, ctx->v32.as<float>(), y, ntiles, int(nrb), jsplit, tps, stride); break;
        case 6: launch_f32_s<6>(c, grid, s, js, is, ctx->v32.as<float>(), y, ntiles, int(nrb), jsplit, tps, stride); break;
        case 7: launch_f32_s<7>(c, grid, s, js, is, ctx->v32.as<float>(), y, ntiles, int(nrb), jsplit, tps, stride); break;
        case 8: launch_f32_s<8>(c, grid, s, js, is, ctx->v32.as<float>(), y, ntiles, int(nrb), jsplit, tps, stride); break;
        case 9: launch_f32_s<9>(c, grid, s, js, is, ctx->v32.as<float>(), y, ntiles, int(nrb), jsplit, tps, stride); break;
        default: fail(PKM_ERR_UNSUPPORTED, "FP32 product: d must be <= 34");
    }
    PKM_CHECK_LAUNCH();
    if (t0) {
        const double pairs = double(P.n) * double(P.n);
        timing_stop(ctx, t0, PKM_FP32, pairs, pairs * (2.0 * P.d + 2.0 * k));
    }
    return F32Out{y, jsplit, stride, KP};
}

// ---------------------------------------------------------------------------
// FP64 kernel: direct differences on the vector ALUs
// ---------------------------------------------------------------------------
template <int DP, int KC>
__global__ __launch_bounds__(256) void k_mvm_f64(const double* __restrict__ xs, int d,
                                                 const double* __restrict__ V, int64_t ldv,
                                                 int col0, int kcols, int64_t n,
                                                 double sigma2, double* __restrict__ part,
                                                 int64_t ldp, int64_t split_stride,
                                                 int64_t j_per_split) {
    constexpr int JT = 64;
    __shared__ double sx[JT][DP];
    __shared__ double sv[JT][KC];
    const int64_t i = blockIdx.x * int64_t(256) + threadIdx.x;
    const int split = blockIdx.y;
    const int64_t j0 = split * j_per_split;
    const int64_t j1 = min(n, j0 + j_per_split);
    double xi[DP];
#pragma unroll
    for (int r = 0; r < DP; ++r) xi[r] = (i < n && r < d) ? xs[i * d + r] : 0.0;
    double acc[KC];
#pragma unroll
    for (int c = 0; c < KC; ++c) acc[c] = 0.0;
    const double ls2 = log(sigma2);
    for (int64_t jb = j0; jb < j1; jb += JT) {
        __syncthreads();
        for (int e = threadIdx.x; e < JT * DP; e += 256) {
            int jj = e / DP, r = e % DP;
            int64_t j = jb + jj;
            sx[jj][r] = (j < j1 && r < d) ? xs[j * d + r] : 0.0;
        }
        for (int e = threadIdx.x; e < JT * KC; e += 256) {
            int jj = e / KC, c = e % KC;
            int64_t j = jb + jj;
            sv[jj][c] = (j < j1 && col0 + c < kcols) ? V[j * ldv + col0 + c] : 0.0;
        }
        __syncthreads();
        const int jn = int(min<int64_t>(JT, j1 - jb));
        for (int jj = 0; jj < jn; ++jj) {
            double s = 0.0;
#pragma unroll
            for (int r = 0; r < DP; ++r) {
                double t = xi[r] - sx[jj][r];
                s = fma(t, t, s);
            }
            const double kij = exp(fma(-0.5, s, ls2));
#pragma unroll
            for (int c = 0; c < KC; ++c) acc[c] = fma(kij, sv[jj][c], acc[c]);
        }
    }
    if (i < n) {
        double* po = part + split * split_stride + i * ldp + col0;
#pragma unroll
        for (int c = 0; c < KC; ++c)
            if (col0 + c < kcols) po[c] = acc[c];
    }
}

// FP64 product on 16x16x4 FP64 MFMA, same structure as the FP32 one: per
// 16-row j-tile, the exponent tile S^T = B_J A_I^T (S4 MFMAs over the
// augmented operands) leaves lane l with S[i = l % 16][j = l / 16 + 4 r],
// r = 0..3 -- exactly the A operands of four K V MFMAs whose B operands are
// V[j0 + 4 r + l / 16][16 q + l % 16].  exp2 runs on the vector ALUs in
// FP64 (exp2_tab).  Wave: U i-tiles of 16 rows; grid.y splits the j tiles.
// KR = 1: one column past the KT MFMA tiles (k = 16 KT + 1, e.g. a target
// and 16 probes) is summed on the vector ALUs -- four FP64 FMAs per lane and
// tile against the four MFMAs a further 16-column tile would cost on this
// matrix-core-bound kernel -- and reduced across the four lanes of a row
// (l % 16 equal) at the end.
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <int S4, int KT, int U, int KR = 0>
__global__ __launch_bounds__(256) void k_mvm_f64x(const double* __restrict__ jside,
                                                  const double* __restrict__ iside,
                                                  const double* __restrict__ V, int64_t ldv,
                                                  int kcols, int64_t n, int64_t ntiles,
                                                  int64_t n_out,
                                                  double* __restrict__ part, int64_t ldp,
                                                  int64_t split_stride, int64_t tiles_per_split) {
    __shared__ double tab[64];
    if (threadIdx.x < 64) tab[threadIdx.x] = exp2(double(threadIdx.x) / 64.0);
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int g = lane >> 4, cc = lane & 15;
    const int64_t itile0 = (int64_t(blockIdx.x) * 4 + w) * U;
    const int64_t t0 = int64_t(blockIdx.y) * tiles_per_split;
    const int64_t t1 = min(ntiles, t0 + tiles_per_split);
    double ai[U][S4];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
        for (int q = 0; q < S4; ++q) ai[u][q] = iside[((itile0 + u) * 64 + lane) * S4 + q];
    f64x4 acc[U][KT];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
        for (int q = 0; q < KT; ++q) acc[u][q] = f64x4{0.0, 0.0, 0.0, 0.0};
    double racc[U];
#pragma unroll
    for (int u = 0; u < U; ++u) racc[u] = 0.0;
    for (int64_t t = t0; t < t1; ++t) {
        double bj[S4];
#pragma unroll
        for (int q = 0; q < S4; ++q) bj[q] = jside[(t * 64 + lane) * S4 + q];
        double vb[KT][4], vr[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t j = t * 16 + 4 * r + g;
#pragma unroll
            for (int q = 0; q < KT; ++q) {
                const int c = 16 * q + cc;
                vb[q][r] = (j < n && c < kcols) ? V[j * ldv + c] : 0.0;
            }
            if (KR) vr[r] = j < n ? V[j * ldv + 16 * KT] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            f64x4 st = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int q = 0; q < S4; ++q)
                st = __builtin_amdgcn_mfma_f64_16x16x4f64(bj[q], ai[u][q], st, 0, 0, 0);
            double kv[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) kv[r] = exp2_tab(st[r], tab);
#pragma unroll
            for (int q = 0; q < KT; ++q)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    acc[u][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(kv[r], vb[q][r], acc[u][q], 0, 0, 0);
            if (KR) {
#pragma unroll
                for (int r = 0; r < 4; ++r) racc[u] = fma(kv[r], vr[r], racc[u]);
            }
        }
    }
    // FP64 16x16x4 results: lane l holds rows l / 16 + 4 r, column l % 16
    double* po = part + blockIdx.y * split_stride;
    if (KR) {   // lane l holds row l % 16's sum over the j with j % 4 = l / 16
#pragma unroll
        for (int u = 0; u < U; ++u) {
            double v = racc[u];
            v += __shfl_xor(v, 16);
            v += __shfl_xor(v, 32);
            const int64_t i = (itile0 + u) * 16 + cc;
            if (g == 0 && i < n_out) po[i * ldp + 16 * KT] = v;
        }
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
        for (int q = 0; q < KT; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t i = (itile0 + u) * 16 + g + 4 * r;
                const int c = 16 * q + cc;
                if (i < n_out && c < kcols) po[i * ldp + c] = acc[u][q][r];
            }
}

// i-tiles of 16 rows per wave of the FP64 product: four (more independent
// MFMA chains per wave; 5-7 % faster than two at both bench sizes) while the
// augmented length keeps the registers within two waves per SIMD, else two.
template <int S4>
constexpr int kF64xTiles = S4 <= 6 ? 4 : 2;

static int f64x_tiles(int s4) { return s4 <= 6 ? 4 : 2; }

template <int S4>
static void launch_f64x(int KT, dim3 grid, hipStream_t s, const double* js, const double* is,
                        const double* V, int64_t ldv, int k, int64_t n, int64_t ntiles, int64_t n_out,
                        double* part, int64_t ldp, int64_t sstride, int64_t tps) {
    if (k % 16 == 1 && k > 16) {   // KT MFMA tiles and one column on the vector ALUs
        switch (k / 16) {
            case 1: k_mvm_f64x<S4, 1, kF64xTiles<S4>, 1><<<grid, 256, 0, s>>>(js, is, V, ldv, k, n, ntiles, n_out, part, ldp, sstride, tps); return;
            case 2: k_mvm_f64x<S4, 2, kF64xTiles<S4>, 1><<<grid, 256, 0, s>>>(js, is, V, ldv, k, n, ntiles, n_out, part, ldp, sstride, tps); return;
            case 3: k_mvm_f64x<S4, 3, kF64xTiles<S4>, 1><<<grid, 256, 0, s>>>(js, is, V, ldv, k, n, ntiles, n_out, part, ldp, sstride, tps); return;
            default: break;
        }
    }
    switch (KT) {
        case 1: k_mvm_f64x<S4, 1, kF64xTiles<S4>><<<grid, 256, 0, s>>>(js, is, V, ldv, k, n, ntiles, n_out, part, ldp, sstride, tps); break;
        case 2: k_mvm_f64x<S4, 2, kF64xTiles<S4>><<<grid, 256, 0, s>>>(js, is, V, ldv, k, n, ntiles, n_out, part, ldp, sstride, tps); break;
        case 3: k_mvm_f64x<S4, 3, kF64xTiles<S4>><<<grid, 256, 0, s>>>(js, is, V, ldv, k, n, ntiles, n_out, part, ldp, sstride, tps); break;
        case 4: k_mvm_f64x<S4, 4, kF64xTiles<S4>><<<grid, 256, 0, s>>>(js, is, V, ldv, k, n, ntiles, n_out, part, ldp, sstride, tps); break;
        default: fail(PKM_ERR_UNSUPPORTED, "FP64 MFMA product: bad column tiling");
    }
}

template <int DP>
static void launch_f64_d(int kc, dim3 grid, hipStream_t s, const double* xs, int d,
                         const double* V, int64_t ldv, int col0, int k, int64_t n,
                         double sigma2, double* part, int64_t ldp, int64_t sstride,
                         int64_t jps) {
#define PKM_F64_CASE(KC)                                                                 \
    case KC:                                                                             \
        k_mvm_f64<DP, KC><<<grid, 256, 0, s>>>(xs, d, V, ldv, col0, k, n, sigma2, part, \
                                                ldp, sstride, jps);                      \
        break;
    switch (kc) {
        PKM_F64_CASE(1) PKM_F64_CASE(2) PKM_F64_CASE(4) PKM_F64_CASE(8)
        PKM_F64_CASE(12) PKM_F64_CASE(17) PKM_F64_CASE(24)
        default: fail(PKM_ERR_UNSUPPORTED, "FP64 product: bad column chunk");
    }
#undef PKM_F64_CASE
}

// Sum of split partials (FP64), written to Y with leading dimension ldy.
__global__ void k_sum_splits64(const double* __restrict__ part, int nsplit, int64_t sstride,
                               int64_t n, int k, int64_t ldp, double* __restrict__ Y,
                               int64_t ldy) {
    int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (e >= n * k) return;
    int64_t i = e / k;
    int c = int(e - i * k);
    double s = 0.0;
    for (int p = 0; p < nsplit; ++p) s += part[p * sstride + i * ldp + c];
    Y[i * ldy + c] = s;
}

void mvm_k64(pkm_ctx* ctx, int k, const double* V, int ldv, double* Y, int ldy) {
    Prepared& P = ctx->P();
    PKM_REQUIRE(P.valid64, "internal: FP64 operands not prepared");
    hipStream_t s = ctx->stream;
    const int64_t n = P.n;
    const int d = P.d;
    const bool use_mfma = P.d4 <= kAug64MaxD4 && k >= 4;
    // rows per work-group: 4 waves x f64x_tiles x 16 on the MFMA path, 256 otherwise
    const int64_t rows_wg = use_mfma ? 64 * f64x_tiles(P.d4 / 4) : 256;
    int64_t nrb = cdiv(n, rows_wg);
    int jsplit = 1;
    while (jsplit < 64 && nrb * jsplit < 2048 && n / (jsplit * 2) >= 256) jsplit <<= 1;
    int64_t jps = round_up(cdiv(n, jsplit), 64);
    jsplit = int(cdiv(n, jps));
    int64_t sstride = n * int64_t(k);
    ctx->y64pad.ensure(sizeof(double) * sstride * jsplit);
    double* part = ctx->y64pad.as<double>();
    dim3 grid((unsigned)(nrb), (unsigned)(jsplit));

    const hipEvent_t t0 = ctx->timing ? timing_start(ctx) : nullptr;
    const double* xs = P.xs64.as<double>();
    if (use_mfma) {
        // j tiles of 16 rows over the padded length; jps is a multiple of 64
        const int64_t ntiles = P.n_pad / 16;
        const int64_t tps = jps / 16;
        const double* js = P.jside64.as<double>();
        const double* is = P.iside64.as<double>();
        for (int col0 = 0; col0 < k; col0 += 64) {
            const int kc = std::min(64, k - col0);
            const int KT = int(cdiv(kc, 16));
            switch (P.d4 / 4) {
#define PKM_F64X(S4)                                                                          \
    case S4:                                                                                  \
        launch_f64x<S4>(KT, grid, s, js, is, V + col0, ldv, kc, n, ntiles, n, part + col0, k, \
                        sstride, tps);                                                        \
        break;
                PKM_F64X(1) PKM_F64X(2) PKM_F64X(3) PKM_F64X(4) PKM_F64X(5)
                PKM_F64X(6) PKM_F64X(7) PKM_F64X(8) PKM_F64X(9)
#undef PKM_F64X
                default: fail(PKM_ERR_UNSUPPORTED, "FP64 MFMA product: augmented length");
            }
            PKM_CHECK_LAUNCH();
        }
    } else {
        for (int col0 = 0; col0 < k;) {
            int rem = k - col0;
            int kc;
            if (rem > 24) kc = 24;
            else if (rem > 17) kc = 24;
            else if (rem > 12) kc = 17;
            else if (rem > 8) kc = 12;
            else if (rem > 4) kc = 8;
            else if (rem > 2) kc = 4;
            else kc = rem;
            if (d <= 4) launch_f64_d<4>(kc, grid, s, xs, d, V, ldv, col0, k, n, P.sigma2, part, k, sstride, jps);
            else if (d <= 8) launch_f64_d<8>(kc, grid, s, xs, d, V, ldv, col0, k, n, P.sigma2, part, k, sstride, jps);
            else if (d <= 16) launch_f64_d<16>(kc, grid, s, xs, d, V, ldv, col0, k, n, P.sigma2, part, k, sstride, jps);
            else if (d <= 32) launch_f64_d<32>(kc, grid, s, xs, d, V, ldv, col0, k, n, P.sigma2, part, k, sstride, jps);
            else launch_f64_d<64>(kc, grid, s, xs, d, V, ldv, col0, k, n, P.sigma2, part, k, sstride, jps);
            PKM_CHECK_LAUNCH();
            col0 += kc;
        }
    }
    if (t0) {
        const double pairs = double(n) * double(n);
        timing_stop(ctx, t0, PKM_FP64, pairs, pairs * (2.0 * d + 2.0 * k));
    }
    int64_t tot = n * k;
    k_sum_splits64<<<cdiv(tot, 256), 256, 0, s>>>(part, jsplit, sstride, n, k, k, Y, ldy);
    PKM_CHECK_LAUNCH();
}

void cross_k64(pkm_ctx* ctx, const pkm_problem* prob, const double* Xa, int64_t na,
               const double* Xb, int64_t nb, int k, const double* V, double* Y) {
    hipStream_t s = ctx->stream;
    const int d4 = int(round_up(prob->d + 2, 4));
    PKM_REQUIRE(d4 <= kAug64MaxD4, "cross product needs d <= 34");
    const int64_t nap = round_up(na, 256), nbp = round_up(nb, 256);
    ctx->cross[0].ensure(sizeof(double) * nbp * d4);
    ctx->cross[1].ensure(sizeof(double) * nap * d4);
    ctx->cross[2].ensure(sizeof(double) * std::max(nap, nbp) * d4);
    double* js = ctx->cross[0].as<double>();
    double* is = ctx->cross[1].as<double>();
    prepare_cross64(ctx, prob, Xa, na, Xb, nb, js, is, ctx->cross[2].as<double>());
    const int64_t nrb = cdiv(na, 64 * f64x_tiles(d4 / 4));
    int jsplit = 1;
    while (jsplit < 64 && nrb * jsplit < 2048 && nb / (jsplit * 2) >= 256) jsplit <<= 1;
    const int64_t jps = round_up(cdiv(nb, jsplit), 64);
    jsplit = int(cdiv(nb, jps));
    const int64_t sstride = na * int64_t(k);
    ctx->y64pad.ensure(sizeof(double) * sstride * jsplit);
    double* part = ctx->y64pad.as<double>();
    const dim3 grid((unsigned)nrb, (unsigned)jsplit);
    const int64_t ntiles = nbp / 16, tps = jps / 16;
    for (int col0 = 0; col0 < k; col0 += 64) {
        const int kc = std::min(64, k - col0);
        const int KT = int(cdiv(kc, 16));
        switch (d4 / 4) {
#define PKM_F64C(S4)                                                                            \
    case S4:                                                                                    \
        launch_f64x<S4>(KT, grid, s, js, is, V + col0, k, kc, nb, ntiles, na, part + col0, k, \
                        sstride, tps);                                                          \
        break;
            PKM_F64C(1) PKM_F64C(2) PKM_F64C(3) PKM_F64C(4) PKM_F64C(5)
            PKM_F64C(6) PKM_F64C(7) PKM_F64C(8) PKM_F64C(9)
#undef PKM_F64C
            default: fail(PKM_ERR_UNSUPPORTED, "cross product: augmented length");
        }
        PKM_CHECK_LAUNCH();
    }
    k_sum_splits64<<<cdiv(na * k, 256), 256, 0, s>>>(part, jsplit, sstride, na, k, k, Y, k);
    PKM_CHECK_LAUNCH();
}

// Y = sum_splits(part32) + lambda V, FP64 out.
// (zero_after: the column-maxima slots cleared for the next product, by the
// first work-group)
__global__ void k_finish32(const float* __restrict__ part, int nsplit, int64_t sstride, int kp,
                           int64_t n, int k, const double* __restrict__ V, int64_t ldv,
                           double lambda, double* __restrict__ Y, int64_t ldy,
                           unsigned long long* __restrict__ zero_after) {
    int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (zero_after && e < kColmaxSlots) zero_after[e] = 0ull;
    if (e >= n * k) return;
    int64_t i = e / k;
    int c = int(e - i * k);
    double s = 0.0;
    for (int p = 0; p < nsplit; ++p) s += double(part[p * sstride + i * kp + c]);
    Y[i * ldy + c] = s + lambda * V[i * ldv + c];
}

__global__ void k_axpy_lam(int64_t n, int k, const double* __restrict__ V, double lambda,
                           double* __restrict__ Y) {
    int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (e >= n * k) return;
    Y[e] += lambda * V[e];
}

void mvm(pkm_ctx* ctx, int prec, int k, const double* V, double* Y) {
    mvm_shift(ctx, prec, k, V, Y, ctx->P().lambda);
}

void mvm_shift(pkm_ctx* ctx, int prec, int k, const double* V, double* Y, double shift) {
    Prepared& P = ctx->P();
    hipStream_t s = ctx->stream;
    const int64_t n = P.n;
    if (prec == PKM_FP64) {
        mvm_k64(ctx, k, V, k, Y, k);
        k_axpy_lam<<<cdiv(n * k, 256), 256, 0, s>>>(n, k, V, shift, Y);
        PKM_CHECK_LAUNCH();
        return;
    }
    if (prec == PKM_I8X) {
        mvm_i8(ctx, k, V, k, Y, k, shift);
        return;
    }
    PKM_REQUIRE(prec == PKM_FP32 || prec == PKM_BF16X1 || prec == PKM_BF16X3 || prec == PKM_F16X3,
                "unknown precision");
    // FP32 products take up to 65 columns per pass, 16-bit ones up to seven
    // tiles; a wider block is split into passes of equal width (k = 129 as
    // 65 + 64: 3.62 ms at 65,536 points against 3.85 ms as 112 + 17)
    const int kmax = prec == PKM_FP32 ? 65 : kBf16MaxCols;
    const int npass = int(cdiv(k, kmax));
    const int width = int(cdiv(k, npass));
    for (int c0 = 0; c0 < k; c0 += width) {
        int kc = std::min(width, k - c0);
        F32Out o = prec == PKM_FP32 ? mvm_k32(ctx, kc, V + c0, k)
                                    : mvm_kbf16(ctx, prec, kc, V + c0, k);
        k_finish32<<<cdiv(n * kc, 256), 256, 0, s>>>(o.y, o.jsplit, o.stride, o.kp, n, kc, V + c0, k,
                                                      shift, Y + c0, k, o.zero_after);
        PKM_CHECK_LAUNCH();
        if (o.zero_after) ctx->colmax_clean = true;
    }
}

}  // namespace pkm
