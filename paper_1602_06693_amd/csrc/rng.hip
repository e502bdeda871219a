// Rademacher probes on the device from the SplitMix64 generator (Steele, Lea
// and Flood, OOPSLA 2014; finaliser of the reference splitmix64.c), for the
// stochastic trace estimate of Section 2.1.  Seeded with s, output number t
// (t >= 1) is mix(s + t * GAMMA mod 2^64), so every element is computed from
// its own counter: element (i, c) of an n x ncols block takes t = i ncols + c
// + 1 and is -1 when the output's top bit is set, else +1.
#include "pkm_internal.h"

namespace pkm {

__device__ inline uint64_t splitmix64_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// one thread per row segment of up to 64 columns: the row index is the
// block's, the column the thread's (no 64-bit division per element)
__global__ __launch_bounds__(256) void k_rademacher(int64_t n, int ncols, uint64_t seed,
                                                    double* __restrict__ Z, int64_t ldz) {
    const int64_t i = blockIdx.x * int64_t(4) + (threadIdx.x >> 6);
    if (i >= n) return;
    for (int c = threadIdx.x & 63; c < ncols; c += 64) {
        const uint64_t t = uint64_t(i) * uint64_t(ncols) + uint64_t(c) + 1ull;
        const uint64_t z = splitmix64_mix(seed + t * 0x9E3779B97F4A7C15ull);
        Z[i * ldz + c] = (z >> 63) ? -1.0 : 1.0;
    }
}

void rademacher(pkm_ctx* ctx, int64_t n, int ncols, uint64_t seed, double* Z, int64_t ldz) {
    k_rademacher<<<cdiv(n, 4), 256, 0, ctx->stream>>>(n, ncols, seed, Z, ldz);
    PKM_CHECK_LAUNCH();
}

}  // namespace pkm
