// Allocation-free kernel product (pkm_kernel_mvm_noalloc): the PKM_I8X
// product of mvm_i8.hip with every scratch byte in one file-scope device
// array, for callers that cannot allocate device memory (code under HIP graph
// capture, tight serving loops, harnesses that forbid hipMalloc).
//
// The array's address differs per device and is looked up once per device at
// context creation (pkm_create, with that device current); host code uses
// that pointer only -- in host code the array's name is a host-side stand-in,
// not a device address.  Every call on a device shares the array, so calls
// that overlap on one device (several streams or contexts) race; each call
// rewrites all of the scratch it reads.

#include "pkm_internal.h"
#include "i8_internal.h"

#include <algorithm>
#include <mutex>
#include <string>

namespace pkm {

constexpr size_t kNoAllocBytes = size_t(128) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

void noalloc_init(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    PKM_REQUIRE(device >= 0 && device < kMaxDevices, "device index out of range");
    if (g_scratch_ptr[device]) return;
    void* ptr = nullptr;
    PKM_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    PKM_REQUIRE(ptr != nullptr, "scratch symbol has no device address");
    g_scratch_ptr[device] = ptr;
}

size_t noalloc_capacity() { return kNoAllocBytes; }

// 1 / l_r by value (no host-to-device copy) and the column means of X, into
// consts[0..63] and consts[64..127].
struct InvL {
    double v[64];
};
__global__ void k_noalloc_consts(InvL inv_l, const double* __restrict__ X, int64_t n, int d,
                                 double* __restrict__ consts) {
    __shared__ double sh[256];
    const int r = blockIdx.x;
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) acc += X[i * d + r];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        consts[r] = inv_l.v[r];
        consts[64 + r] = sh[0] / double(n);
    }
}

// Y = (K + shift I) V with the PKM_I8X arithmetic and launch shapes of
// mvm_i8 (so results equal pkm_kernel_mvm's bit for bit), all scratch carved
// from the static array: constants, prepared operands, and (reused by every
// column group) maxima, packed digits and partial planes.  Fails
// (PKM_ERR_INVALID) when that does not fit.
void mvm_i8_noalloc(pkm_ctx* ctx, const pkm_problem* prob, int k, const double* V, double* Y,
                    double shift) {
    void* base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        PKM_REQUIRE(ctx->device >= 0 && ctx->device < kMaxDevices, "device index out of range");
        base = g_scratch_ptr[ctx->device];
    }
    PKM_REQUIRE(base != nullptr, "scratch not initialised for this device");
    PKM_REQUIRE(prob->d <= 32, "int8-digit product supports d <= 32");
    const int64_t n = prob->n, n_pad = round_up(n, 256);
    const int d = prob->d, dq = int(round_up(d, 4));
    size_t need_group = 0;
    for (int c0 = 0; c0 < k; c0 += 33) {
        const int kc = std::min(33, k - c0);
        const I8Shape h = i8_shape(n, n_pad, kc);
        need_group = std::max(need_group, kI8CmBytes + i8_vb_bytes(h) + i8_vl_bytes(h) +
                                              i8_part_bytes(h, n, kc));
    }
    const size_t b_consts = 256 * sizeof(double);
    const size_t b_x = round_up(sizeof(double) * size_t(n_pad) * dq, 256);
    const size_t b_ni = round_up(sizeof(double) * size_t(n_pad), 256);
    const size_t b_njl = sizeof(double) * size_t(n_pad) * 16;
    const size_t need = b_consts + 2 * b_x + b_ni + b_njl + need_group;
    if (need > kNoAllocBytes)
        fail(PKM_ERR_INVALID, "pkm_kernel_mvm_noalloc: n = " + std::to_string(n) + ", d = " +
                                  std::to_string(d) + ", k = " + std::to_string(k) + " needs " +
                                  std::to_string(need >> 20) + " MiB of scratch; the limit is " +
                                  std::to_string(kNoAllocBytes >> 20) + " MiB");
    char* at = static_cast<char*>(base);
    double* consts = reinterpret_cast<double*>(at);
    at += b_consts;
    double* xj = reinterpret_cast<double*>(at);
    at += b_x;
    double* xi = reinterpret_cast<double*>(at);
    at += b_x;
    double* ni = reinterpret_cast<double*>(at);
    at += b_ni;
    double* njl = reinterpret_cast<double*>(at);
    at += b_njl;
    char* group_base = at;

    hipStream_t s = ctx->stream;
    InvL il{};
    for (int r = 0; r < d; ++r) il.v[r] = 1.0 / prob->lengthscales[r];
    k_noalloc_consts<<<d, 256, 0, s>>>(il, prob->X, n, d, consts);
    PKM_CHECK_LAUNCH();
    i8_prepare_into(s, prob->X, n, d, consts, consts + 64, xj, xi, ni, njl);
    const I8Prep P{xj, xi, njl, ni, n, n_pad, d, dq, prob->sigma2};
    i8_check_prep(P, b_x, b_x, b_ni, b_njl);
    for (int c0 = 0; c0 < k;) {
        const int kc = std::min(33, k - c0);
        const I8Shape h = i8_shape(n, n_pad, kc);
        char* g = group_base;
        I8Work w;
        w.bm = reinterpret_cast<double*>(g);
        w.ex = reinterpret_cast<int*>(w.bm + 64 * 64);
        g += kI8CmBytes;
        w.vb = reinterpret_cast<uint32_t*>(g);
        g += i8_vb_bytes(h);
        w.vl = reinterpret_cast<uint32_t*>(g);
        g += i8_vl_bytes(h);
        w.part = reinterpret_cast<double*>(g);
        i8_run_group(nullptr, s, P, h, w, kc, V + c0, k, Y + c0, k, shift);
        c0 += kc;
    }
}

}  // namespace pkm
