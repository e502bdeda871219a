// FP64-class kernel product on int8 matrix cores (PKM_I8X).
//
// Where lambda is small against |K| (Section 2.1's K_y = K + lambda I with
// smooth kernels), a product whose error is not far below lambda / |K| leaves
// the PCG recursion and the FP64 true residual apart, and FP32-class
// products never certify.  This product keeps every rounding at 2^-30 of an
// entry's scale and free of row- or column-wise structure:
//
//   exponent   S_ij = 2 xh_i . xh_j - |xh_i|^2 - |xh_j|^2  (log2 of K_ij / sigma2;
//              xh = (x - mean) / l * sqrt(log2(e) / 2)), the cross term on
//              16x16x4 FP64 MFMA (the j norms enter as the accumulator's
//              initial value), the i norm subtracted in FP64;
//   exp2       table-driven in FP64 (S = N / 4096 + r, |r| <= 1/8192;
//              2^(N / 4096) from a 4096-entry LDS table scaled by 2^30; 2^r - 1
//              by its quadratic Taylor polynomial, truncation ~1e-13
//              relative), rounded to the nearest integer kint =
//              rint(2^30 K / sigma2) in [0, 2^30];
//   digits     kint and vint = rint(2^e V) (per column, max |V| 2^e in
//              [2^29, 2^30)) written in signed base-256 digits s_0 .. s_3 in
//              [-128, 127]: x + 0x80808080 has the bytes s_p + 128 (the
//              addition rides on the rounding constant), and XOR 0x80 per byte
//              turns them into the two's-complement bytes s_p;
//   K V        digit pairs (p, q) on 16x16x64 int8 MFMA with exact int32
//              accumulation, one accumulator per weight class c = p + q
//              (c >= 2 kept: 13 of the 16 pairs); the epilogue forms
//              sum_c 256^c G_c in FP64 and scales by sigma2 2^(-30 - e).
//
// Lane layout.  The FP64 exponent tile of j-tile t leaves lane l with
// S[i = l % 16][j = 16 t + l / 16 + 4 r], r = 0..3; over the four j-tiles of a
// 64-row chunk that is 16 values per lane, byte b = 4 t + r of the int8 MFMA A
// operand.  The V digits are packed so that byte b of lane l holds
// V[j = 64 T + 16 (b / 4) + l / 16 + 4 (b % 4)][column l % 16] (A and B of the
// int8 MFMA share the lane-group -> K-index map).  A column k - 1 past KT
// full 16-column tiles (KR = 1) takes one MFMA per K digit: its B operand
// holds the four V digits of that column in tile columns 0..3.
//
// int32 range: a class sums at most 3 pairs of |s_p s_q| <= 2^14 per j, so a
// work-group's j range is at most 32768 rows (the host splits j accordingly).

#include "pkm_internal.h"
#include "i8_internal.h"

#include <algorithm>
#include <cmath>
#include <mutex>

namespace pkm {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int kI8MaxJ = 32768;        // rows of j per work-group (int32 range)
constexpr double kMagic = 6755399441055744.0;                    // 1.5 * 2^52
constexpr double kMagicDig = 6755399441055744.0 + 2155905152.0;  // + 0x80808080

// ---------------------------------------------------------------------------
// preparation: FP64 cross-term operands and row norms
// ---------------------------------------------------------------------------
// One thread per padded row: xj (16 xh) and xi (32 xh) in 16x16x4 lane order
// (tile t, lane l, group s) <-> row 16 t + l % 16, slot 4 s + l / 16, with
// SQ = dq / 4 groups; ni = 4096 |xh_i|^2 (0 for padded rows).  The factor
// 4096 (exact) makes the contraction 4096 S, the form the exp2 rounds in.
__global__ void k_prep_i8(const double* __restrict__ X, int64_t n, int64_t n_pad, int d, int SQ,
                          const double* __restrict__ inv_l, const double* __restrict__ mean,
                          double* __restrict__ xj, double* __restrict__ xi,
                          double* __restrict__ ni) {
    const int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (i >= n_pad) return;
    const double c = sqrt(0.5 * 1.4426950408889634);
    const int64_t t = i >> 4;
    const int row = int(i & 15);
    double nrm = 0.0;
    for (int sl = 0; sl < 4 * SQ; ++sl) {
        double v = 0.0;
        if (i < n && sl < d) v = (X[i * d + sl] - mean[sl]) * inv_l[sl] * c;
        nrm = fma(v, v, nrm);
        const int64_t at = (t * 64 + row + 16 * (sl & 3)) * SQ + (sl >> 2);
        xj[at] = 64.0 * v;
        xi[at] = 128.0 * v;
    }
    ni[i] = 4096.0 * nrm;
}

// Negated j norms in exponent-tile lane order: njl[(t * 64 + l) * 4 + r] =
// -4096 |xh_j|^2 for j = 16 t + l / 16 + 4 r; padded rows get -1e30 (K = 0).
// 256 entries per 16-row tile (each norm repeated for the 16 lanes of its
// lane group): 16 n_pad doubles.
__global__ void k_prep_njl(const double* __restrict__ ni, int64_t n, int64_t n_pad,
                           double* __restrict__ njl) {
    const int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (e >= n_pad * 16) return;
    const int64_t t = e >> 8;
    const int l = int((e >> 2) & 63), r = int(e & 3);
    const int64_t j = 16 * t + l / 16 + 4 * r;
    njl[e] = j < n ? -ni[j] : -1.0e30;
}

void i8_prepare_into(hipStream_t s, const double* X, int64_t n, int d, const double* inv_l,
                     const double* mean, double* xj, double* xi, double* ni, double* njl) {
    const int64_t n_pad = round_up(n, 256);
    const int SQ = int(round_up(d, 4)) / 4;
    k_prep_i8<<<cdiv(n_pad, 256), 256, 0, s>>>(X, n, n_pad, d, SQ, inv_l, mean, xj, xi, ni);
    PKM_CHECK_LAUNCH();
    k_prep_njl<<<cdiv(n_pad * 16, 256), 256, 0, s>>>(ni, n, n_pad, njl);
    PKM_CHECK_LAUNCH();
}

static void prepare_i8(pkm_ctx* ctx) {
    Prepared& P = ctx->P();
    if (P.validi8) return;
    PKM_REQUIRE(P.d <= 32, "int8-digit product supports d <= 32");
    P.dq = int(round_up(P.d, 4));
    P.xj8.ensure(sizeof(double) * P.n_pad * P.dq);
    P.xi8.ensure(sizeof(double) * P.n_pad * P.dq);
    P.ni8.ensure(sizeof(double) * P.n_pad);
    P.njl8.ensure(sizeof(double) * P.n_pad * 16);
    const double* inv_l = ctx->scal.as<double>();
    i8_prepare_into(ctx->stream, P.X, P.n, P.d, inv_l, inv_l + 64, P.xj8.as<double>(),
                    P.xi8.as<double>(), P.ni8.as<double>(), P.njl8.as<double>());
    P.validi8 = true;
}

// ---------------------------------------------------------------------------
// V: column maxima -> exponents, digit packing
// ---------------------------------------------------------------------------
// Per-block largest |V[:, c]|: bm[blockIdx.x * k + c] (grid.y = columns).
__global__ void k_i8_colmax(const double* __restrict__ V, int64_t ldv, int64_t n, int k,
                            double* __restrict__ bm) {
    __shared__ double sh[4];
    const int c = blockIdx.y;
    double m = 0.0;
    for (int64_t j = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; j < n;
         j += int64_t(gridDim.x) * blockDim.x)
        m = fmax(m, fabs(V[j * ldv + c]));
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) bm[int64_t(blockIdx.x) * k + c] = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
}

// e_c with max |V_c| 2^e_c in [2^29, 2^30) from the nb per-block maxima; 0 for
// an all-zero column (and for a non-finite one: V must be finite).
__global__ void k_i8_exps(const double* __restrict__ bm, int nb, int k, int* __restrict__ ex) {
    const int c = threadIdx.x;
    if (c >= k) return;
    double m = 0.0;
    for (int b = 0; b < nb; ++b) m = fmax(m, bm[b * k + c]);
    ex[c] = (m > 0.0 && m <= 1.7976931348623157e308) ? 29 - ilogb(m) : 0;
}

// Digit dword of four values' digit q: byte r = digit q of vals[r].  Values
// arrive offset by 0x80808080 (bytes s_p + 128); the XOR makes the bytes s_p.
__device__ inline uint32_t digit_dword(const uint32_t (&w)[4], int q) {
    uint32_t out = 0;
#pragma unroll
    for (int r = 0; r < 4; ++r) out |= ((w[r] >> (8 * q)) & 0xffu) << (8 * r);
    return out ^ 0x80808080u;
}

// One thread per (chunk T, column tile qt (KT = last column when KR), lane,
// j-tile jt): four rows j = 64 T + 16 jt + lane / 16 + 4 r of column
// 16 qt + lane % 16 -> dword jt of the four digit operands.
//   vb[((T * KT + qt) * 4 + q) * 64 + lane].dword[jt]   full tiles
//   vl[T * 64 + lane].dword[jt]                          last column (q = lane % 16 < 4)
__global__ void k_i8_pack(const double* __restrict__ V, int64_t ldv, int64_t n, int k, int64_t nchunk,
                          int KT, int KR, const int* __restrict__ ex, uint32_t* __restrict__ vb,
                          uint32_t* __restrict__ vl) {
    const int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    const int tiles = KT + KR;
    if (e >= nchunk * tiles * 256) return;
    const int jt = int(e & 3);
    const int lane = int((e >> 2) & 63);
    const int64_t rest = e >> 8;
    const int qt = int(rest % tiles);
    const int64_t T = rest / tiles;
    const int g = lane >> 4, cl = lane & 15;
    const bool last = qt == KT;
    const int col = last ? k - 1 : 16 * qt + cl;
    uint32_t w[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int64_t j = 64 * T + 16 * jt + g + 4 * r;
        double v = 0.0;
        if (j < n && col < k && (!last || cl < 4)) v = V[j * ldv + col];
        const double sv = ldexp(v, ex[col < k ? col : 0]);
        w[r] = uint32_t(__double2loint(sv + kMagicDig));
    }
    if (!last) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
            vb[((((T * KT + qt) * 4 + q) * 64 + lane) << 2) + jt] = digit_dword(w, q);
    } else {
        // tile column cl < 4 carries digit q = cl of column k - 1
        vl[((T * 64 + lane) << 2) + jt] = cl < 4 ? digit_dword(w, cl) : 0u;
    }
}

// ---------------------------------------------------------------------------
// the product kernel
// ---------------------------------------------------------------------------
// 4-value byte transpose: in w[r] byte p = digit p of value r (offset form);
// out[p] byte r = digit p of value r (two's-complement digits).
__device__ inline void transpose_digits(const uint32_t (&w)[4], uint32_t (&out)[4]) {
    // stage 1: pair values (0,1) and (2,1): [a0 b0 a1 b1], [a2 b2 a3 b3] ...
    const uint32_t t0 = __builtin_amdgcn_perm(w[1], w[0], 0x05010400u);
    const uint32_t t1 = __builtin_amdgcn_perm(w[1], w[0], 0x07030602u);
    const uint32_t t2 = __builtin_amdgcn_perm(w[3], w[2], 0x05010400u);
    const uint32_t t3 = __builtin_amdgcn_perm(w[3], w[2], 0x07030602u);
    // stage 2: [a0 b0 c0 d0], [a1 b1 c1 d1], [a2 b2 c2 d2], [a3 b3 c3 d3]
    out[0] = __builtin_amdgcn_perm(t2, t0, 0x05040100u) ^ 0x80808080u;
    out[1] = __builtin_amdgcn_perm(t2, t0, 0x07060302u) ^ 0x80808080u;
    out[2] = __builtin_amdgcn_perm(t3, t1, 0x05040100u) ^ 0x80808080u;
    out[3] = __builtin_amdgcn_perm(t3, t1, 0x07060302u) ^ 0x80808080u;
}

// kint + 0x80808080 (mod 2^32) for kint = rint(2^30 2^S), from S4 = 4096 S
// <= 0 (clamped at -80 x 4096, where the value rounds to 0):
//   N = rint(S4) (through the rounding constant), rr = S4 - N in [-1/2, 1/2],
//   2^S = 2^(N >> 12) 2^((N & 4095) / 4096) 2^(rr / 4096),
// the middle factor from tab[m] = 2^30 2^(m / 4096), the last as 1 + p with
// p = q + q^2 / 2, q = rr ln2 / 4096 (truncation q^3 / 6 < 1.1e-13 relative;
// a 256-entry table needs the cubic term and one more FMA per entry).
// Every FP64 operation takes at most one constant that is not an inline one.
__device__ inline uint32_t kfix_digits(double S4, const double* __restrict__ tab, double c1,
                                       double c2) {
    S4 = fmax(S4, -80.0 * 4096.0);
    const double y = S4 + kMagic;                    // rint(S4) + 1.5 2^52
    const int m = __double2loint(y);
    const double rr = S4 - (y - kMagic);             // exact
    const double p = rr * fma(rr, c2, c1);
    const double T = tab[m & 4095];
    const double kf = ldexp(fma(T, p, T), m >> 12);  // 2^30 2^S
    return uint32_t(__double2loint(kf + kMagicDig));
}

template <int SQ, int KT, int KR, int U>
__global__ __launch_bounds__(256) void k_mvm_i8(
    const double* __restrict__ xj, const double* __restrict__ xi,
    const double* __restrict__ njl, const double* __restrict__ ni,
    const v4i* __restrict__ vb, const v4i* __restrict__ vl, const int* __restrict__ ex,
    double* __restrict__ part, int64_t nchunk, int nrb, int jsplit, int64_t chunks_per_split,
    int64_t split_stride, int64_t n_out, int k, double s2) {
    __shared__ double tab[4096];   // 32 KiB
    for (int e = threadIdx.x; e < 4096; e += 256) tab[e] = ldexp(exp2(double(e) / 4096.0), 30);
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int b = blockIdx.x;
    const int xcd = b & 7, slot = b >> 3;
    const int group = 8 / jsplit;   // jsplit divides 8: one split per XCD group
    const int split = xcd % jsplit;
    const int rb = slot * group + xcd / jsplit;
    if (rb >= nrb) return;
    const int64_t itile0 = (int64_t(rb) * 4 + wave) * U;
    const int g = lane >> 4, cl = lane & 15;
    // polynomial coefficients of 2^(rr / 4096) - 1 in rr (held in registers)
    constexpr double L = 0.6931471805599453 / 4096.0;
    const double c1 = L, c2 = L * L / 2.0;

    double ai[U][SQ], nin[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
        for (int s = 0; s < SQ; ++s) ai[u][s] = xi[((itile0 + u) * 64 + lane) * SQ + s];
        nin[u] = ni[(itile0 + u) * 16 + cl];
    }
    v4i acc[U][KT > 0 ? KT : 1][5];
    v4i accl[U][4];
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
        for (int q = 0; q < (KT > 0 ? KT : 1); ++q)
#pragma unroll
            for (int c = 0; c < 5; ++c) acc[u][q][c] = v4i{0, 0, 0, 0};
#pragma unroll
        for (int p = 0; p < 4; ++p) accl[u][p] = v4i{0, 0, 0, 0};
    }

    const int64_t T0 = int64_t(split) * chunks_per_split;
    const int64_t T1 = min(nchunk, T0 + chunks_per_split);
    // packed V digits of the current chunk; the next chunk's are loaded one
    // chunk ahead (clamped to the last chunk of the range: always in bounds)
    v4i vv[KT > 0 ? KT : 1][4];
    v4i vlast = v4i{0, 0, 0, 0};
    auto load_v = [&](int64_t T, v4i (&dst)[KT > 0 ? KT : 1][4], v4i& dl) {
#pragma unroll
        for (int qt = 0; qt < KT; ++qt)
#pragma unroll
            for (int q = 0; q < 4; ++q) dst[qt][q] = vb[((T * KT + qt) * 4 + q) * 64 + lane];
        if (KR) dl = vl[T * 64 + lane];
    };
    if (T0 < T1) load_v(T0, vv, vlast);
    for (int64_t T = T0; T < T1; ++T) {
        v4i vn[KT > 0 ? KT : 1][4];
        v4i vln = v4i{0, 0, 0, 0};
        load_v(T + 1 < T1 ? T + 1 : T, vn, vln);
        // K digits of this chunk for every i-tile: ka[u][p] dword jt
        uint32_t ka[U][4][4];
#pragma unroll
        for (int jt = 0; jt < 4; ++jt) {
            const int64_t t = 4 * T + jt;
            double bj[SQ];
#pragma unroll
            for (int s = 0; s < SQ; ++s) bj[s] = xj[(t * 64 + lane) * SQ + s];
            const f64x4 nj = *reinterpret_cast<const f64x4*>(njl + (t * 64 + lane) * 4);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                f64x4 st = nj;
#pragma unroll
                for (int s = 0; s < SQ; ++s)
                    st = __builtin_amdgcn_mfma_f64_16x16x4f64(bj[s], ai[u][s], st, 0, 0, 0);
                uint32_t w[4], dg[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) w[r] = kfix_digits(st[r] - nin[u], tab, c1, c2);
                transpose_digits(w, dg);
#pragma unroll
                for (int p = 0; p < 4; ++p) ka[u][p][jt] = dg[p];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            v4i kd[4];
#pragma unroll
            for (int p = 0; p < 4; ++p)
                kd[p] = v4i{int(ka[u][p][0]), int(ka[u][p][1]), int(ka[u][p][2]), int(ka[u][p][3])};
#pragma unroll
            for (int qt = 0; qt < KT; ++qt) {
#pragma unroll
                for (int p = 0; p < 4; ++p)
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int c = p + q;
                        if (c >= 2)
                            acc[u][qt][c - 2] = __builtin_amdgcn_mfma_i32_16x16x64_i8(
                                kd[p], vv[qt][q], acc[u][qt][c - 2], 0, 0, 0);
                    }
            }
            if (KR) {
#pragma unroll
                for (int p = 0; p < 4; ++p)
                    accl[u][p] = __builtin_amdgcn_mfma_i32_16x16x64_i8(kd[p], vlast, accl[u][p], 0, 0, 0);
            }
        }
#pragma unroll
        for (int qt = 0; qt < KT; ++qt)
#pragma unroll
            for (int q = 0; q < 4; ++q) vv[qt][q] = vn[qt][q];
        vlast = vln;
    }

    // epilogue: sum_c 256^c G_c in FP64, times sigma2 2^(-30 - e_col)
    double* po = part + int64_t(split) * split_stride;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int64_t row0 = (itile0 + u) * 16 + 4 * g;
#pragma unroll
        for (int qt = 0; qt < KT; ++qt) {
            const int col = 16 * qt + cl;
            const int e = ex[col < k ? col : 0];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                double y = 0.0;
#pragma unroll
                for (int c = 4; c >= 0; --c) y = fma(y, 256.0, double(acc[u][qt][c][r]));
                const int64_t i = row0 + r;
                if (i < n_out && col < k) po[i * k + col] = s2 * ldexp(y, 16 - 30 - e);
            }
        }
        if (KR) {
            // lane with tile column q = cl < 4 holds sum_j s_p(K) s_q(V) for every p
            const int e = ex[k - 1];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                double y = 0.0;
                if (cl < 4) {
#pragma unroll
                    for (int p = 3; p >= 0; --p)
                        if (p + cl >= 2) y += ldexp(double(accl[u][p][r]), 8 * (p + cl));
                }
                y += __shfl_xor(y, 1);
                y += __shfl_xor(y, 2);
                const int64_t i = row0 + r;
                if (cl == 0 && i < n_out) po[i * k + k - 1] = s2 * ldexp(y, -30 - e);
            }
        }
    }
}

// Y = sum of split partials + shift V (FP64).
__global__ void k_i8_finish(const double* __restrict__ part, int nsplit, int64_t sstride,
                            int64_t n, int k, const double* __restrict__ V, int64_t ldv,
                            double shift, double* __restrict__ Y, int64_t ldy) {
    const int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x;
    if (e >= n * k) return;
    const int64_t i = e / k;
    const int c = int(e - i * k);
    double s = 0.0;
    for (int p = 0; p < nsplit; ++p) s += part[p * sstride + e];
    Y[i * ldy + c] = s + shift * V[i * ldv + c];
}

// ---------------------------------------------------------------------------
// host
// ---------------------------------------------------------------------------
// i-tiles of 16 rows per wave.  One (158 VGPRs, three waves per SIMD) runs the
// 262,144-point, 33-column product in 81.9 ms; two (260 VGPRs with the
// next-chunk digits in flight: one wave per SIMD) in 152 ms.
constexpr int kI8U = 1;

// Operands of one launch (views into the prepared buffers).
struct I8Ops {
    const double *xj, *xi, *njl, *ni;
    int64_t n;
    double s2;
};

template <int SQ, int KT, int KR>
static void launch_i8_u(dim3 grid, hipStream_t s, const I8Ops& o, const v4i* vb, const v4i* vl,
                        const int* ex, double* part, int64_t nchunk, int nrb, int jsplit, int64_t cps,
                        int64_t sstride, int k) {
    k_mvm_i8<SQ, KT, KR, kI8U><<<grid, 256, 0, s>>>(o.xj, o.xi, o.njl, o.ni, vb, vl, ex, part,
                                                     nchunk, nrb, jsplit, cps, sstride, o.n, k,
                                                     o.s2);
}

template <int SQ>
static void launch_i8_s(int KT, int KR, dim3 grid, hipStream_t s, const I8Ops& o, const v4i* vb,
                        const v4i* vl, const int* ex, double* part, int64_t nchunk, int nrb,
                        int jsplit, int64_t cps, int64_t sstride, int k) {
#define PKM_I8_CASE(kt, kr)                                                                   \
    if (KT == kt && KR == kr) {                                                               \
        launch_i8_u<SQ, kt, kr>(grid, s, o, vb, vl, ex, part, nchunk, nrb, jsplit, cps, sstride, k); \
        return;                                                                               \
    }
    PKM_I8_CASE(0, 1) PKM_I8_CASE(1, 0) PKM_I8_CASE(1, 1) PKM_I8_CASE(2, 0) PKM_I8_CASE(2, 1)
#undef PKM_I8_CASE
    fail(PKM_ERR_UNSUPPORTED, "int8-digit product: unsupported column tiling");
}

// Launch shape of one column group (kc <= 33 columns: KT tiles of 16 plus at
// most one single column; a remainder of 2..15 columns pads a tile).
// Work-group = 4 waves x kI8U i-tiles; j split so that every split spans at
// most kI8MaxJ rows (int32 range) and the grid holds enough work-groups;
// jsplit divides 8 (XCD mapping).  Past 8 splits of kI8MaxJ rows
// (n > 262144) the j range is covered by nsuper launches.
I8Shape i8_shape(int64_t n, int64_t n_pad, int kc) {
    I8Shape h{};
    h.KT = kc / 16;
    h.KR = kc % 16;
    if (h.KR > 1) {
        h.KT += 1;
        h.KR = 0;
    }
    h.nb = int(std::min<int64_t>(64, cdiv(n, 256)));
    h.nchunk = n_pad / 64;
    h.nrb = cdiv(n_pad, 64 * kI8U);
    const int64_t max_cps = kI8MaxJ / 64;
    h.jsplit = 1;
    while (h.jsplit < 8 && (cdiv(h.nchunk, h.jsplit) > max_cps ||
                            (h.nrb * h.jsplit < 2048 && h.nchunk / (h.jsplit * 2) >= 8)))
        h.jsplit <<= 1;
    h.per_launch = h.jsplit * max_cps;
    h.nsuper = cdiv(h.nchunk, h.per_launch);
    h.cps = h.nsuper > 1 ? max_cps : cdiv(h.nchunk, h.jsplit);
    const int group = 8 / h.jsplit;
    h.grid = dim3((unsigned)(round_up(h.nrb, group) * h.jsplit));
    h.nparts = int64_t(h.jsplit) * h.nsuper;
    return h;
}

// Scratch of one column group: per-block column maxima (64 x 64 doubles),
// column exponents (64 ints), packed V digits (vb: KT tiles x 4 digits, vl:
// the single column; 16 bytes per lane and chunk), FP64 partial planes.
size_t i8_vb_bytes(const I8Shape& h) { return round_up(size_t(16) * h.nchunk * h.KT * 4 * 64 + 16, 256); }
size_t i8_vl_bytes(const I8Shape& h) { return round_up(size_t(16) * h.nchunk * 64 + 16, 256); }
size_t i8_part_bytes(const I8Shape& h, int64_t n, int kc) {
    return round_up(sizeof(double) * size_t(n) * kc * h.nparts, 256);
}

// Prepared operands (views): xj, njl over all j-tiles, xi, ni over all rows.
// One column group: maxima -> exponents, digit packing, the product
// launch(es), and Y = sum of partial planes + shift V.  ctx only times the
// product launches (NULL: untimed).
void i8_run_group(pkm_ctx* ctx, hipStream_t s, const I8Prep& P, const I8Shape& h,
                         const I8Work& w, int kc, const double* V, int ldv, double* Y, int ldy,
                         double shift) {
    const int KT = h.KT, KR = h.KR;
    k_i8_colmax<<<dim3(unsigned(h.nb), unsigned(kc)), 256, 0, s>>>(V, ldv, P.n, kc, w.bm);
    PKM_CHECK_LAUNCH();
    k_i8_exps<<<1, 64, 0, s>>>(w.bm, h.nb, kc, w.ex);
    PKM_CHECK_LAUNCH();
    const int64_t tot = h.nchunk * (KT + KR) * 256;
    k_i8_pack<<<cdiv(tot, 256), 256, 0, s>>>(V, ldv, P.n, kc, h.nchunk, KT, KR, w.ex, w.vb, w.vl);
    PKM_CHECK_LAUNCH();
    const int SQ = P.dq / 4;
    const int64_t sstride = P.n * int64_t(kc);
    const hipEvent_t t0 = ctx && ctx->timing ? timing_start(ctx) : nullptr;
    for (int64_t sp = 0; sp < h.nsuper; ++sp) {
        const int64_t c0 = sp * h.per_launch;
        const int64_t nch = std::min<int64_t>(h.nchunk - c0, h.per_launch);
        // the j operands of this range start at j-tile 4 c0
        const I8Ops o{P.xj + c0 * 4 * 64 * SQ, P.xi, P.njl + c0 * 4 * 64 * 4, P.ni, P.n, P.s2};
        const v4i* vb = reinterpret_cast<const v4i*>(w.vb) + c0 * KT * 4 * 64;
        const v4i* vl = reinterpret_cast<const v4i*>(w.vl) + c0 * 64;
        double* pp = w.part + sp * h.jsplit * sstride;
        switch (SQ) {
#define PKM_I8_SQ(sq)                                                                              \
    case sq:                                                                                       \
        launch_i8_s<sq>(KT, KR, h.grid, s, o, vb, vl, w.ex, pp, nch, int(h.nrb), h.jsplit, h.cps, \
                        sstride, kc);                                                              \
        break;
            PKM_I8_SQ(1) PKM_I8_SQ(2) PKM_I8_SQ(3) PKM_I8_SQ(4)
            PKM_I8_SQ(5) PKM_I8_SQ(6) PKM_I8_SQ(7) PKM_I8_SQ(8)
#undef PKM_I8_SQ
            default: fail(PKM_ERR_UNSUPPORTED, "int8-digit product: d must be <= 32");
        }
        PKM_CHECK_LAUNCH();
    }
    if (t0) {
        const double pairs = double(P.n) * double(P.n);
        timing_stop(ctx, t0, PKM_I8X, pairs, pairs * (2.0 * P.d + 2.0 * kc));
    }
    k_i8_finish<<<cdiv(P.n * kc, 256), 256, 0, s>>>(w.part, int(h.nparts), sstride, P.n, kc, V,
                                                    ldv, shift, Y, ldy);
    PKM_CHECK_LAUNCH();
}

// Extents the kernels index, checked against the buffers: j-tiles
// 4 nchunk = n_pad / 16 (xj: 64 SQ, njl: 256 doubles per tile), i-tiles
// 4 kI8U nrb (xi: 64 SQ doubles, ni: 16 per tile).
void i8_check_prep(const I8Prep& P, size_t xj, size_t xi, size_t ni, size_t njl) {
    const int64_t jtiles = P.n_pad / 16;
    const int SQ = P.dq / 4;
    PKM_REQUIRE(P.n_pad % 256 == 0 && xj >= sizeof(double) * size_t(jtiles) * 64 * SQ &&
                    njl >= sizeof(double) * size_t(jtiles) * 256 &&
                    xi >= sizeof(double) * size_t(jtiles) * 64 * SQ &&
                    ni >= sizeof(double) * size_t(jtiles) * 16,
                "internal: int8 product operand extents");
}

void mvm_i8(pkm_ctx* ctx, int k, const double* V, int ldv, double* Y, int ldy, double shift) {
    prepare_i8(ctx);
    Prepared& Q = ctx->P();
    const I8Prep P{Q.xj8.as<double>(), Q.xi8.as<double>(), Q.njl8.as<double>(), Q.ni8.as<double>(),
                   Q.n, Q.n_pad, Q.d, Q.dq, Q.sigma2};
    i8_check_prep(P, Q.xj8.bytes, Q.xi8.bytes, Q.ni8.bytes, Q.njl8.bytes);
    for (int c0 = 0; c0 < k;) {
        // groups of 33 columns (two tiles and one single column), then the rest
        const int kc = std::min(33, k - c0);
        const I8Shape h = i8_shape(P.n, P.n_pad, kc);
        const size_t vbb = i8_vb_bytes(h), vlb = i8_vl_bytes(h);
        ctx->i8cm.ensure(kI8CmBytes);
        ctx->i8v.ensure(vbb + vlb);
        ctx->i8part.ensure(i8_part_bytes(h, P.n, kc));
        I8Work w;
        w.bm = ctx->i8cm.as<double>();
        w.ex = reinterpret_cast<int*>(w.bm + 64 * 64);
        w.vb = ctx->i8v.as<uint32_t>();
        w.vl = reinterpret_cast<uint32_t*>(ctx->i8v.as<char>() + vbb);
        w.part = ctx->i8part.as<double>();
        i8_run_group(ctx, ctx->stream, P, h, w, kc, V + c0, ldv, Y + c0, ldy, shift);
        c0 += kc;
    }
}

}  // namespace pkm
