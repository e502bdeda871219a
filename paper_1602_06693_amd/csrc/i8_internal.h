// Shared pieces of the int8-digit product (mvm_i8.hip) for the translation
// units that run it with their own scratch.
#pragma once

#include "pkm_internal.h"

namespace pkm {

// Launch shape of one column group (kc <= 33 columns: KT tiles of 16 plus at
// most one single column; a remainder of 2..15 columns pads a tile).
// Work-group = 4 waves x 1 i-tile of 16 rows; j split so that every split
// spans at most 32768 rows (int32 range of the digit sums) and the grid holds
// enough work-groups; jsplit divides 8 (XCD mapping).  Past 8 such splits
// (n > 262144) the j range is covered by nsuper launches.
struct I8Shape {
    int KT, KR, jsplit, nb;
    int64_t nchunk, nrb, nsuper, per_launch, cps, nparts;
    dim3 grid;
};

// Scratch of one column group: per-block column maxima (64 x 64 doubles),
// column exponents (64 ints) -- kI8CmBytes in all --, packed V digits (vb: KT
// tiles x 4 digits, vl: the single column; 16 bytes per lane and chunk), and
// the FP64 partial planes.
struct I8Work {
    double* bm;
    int* ex;
    uint32_t *vb, *vl;
    double* part;
};

constexpr size_t kI8CmBytes = 33024;   // 64 x 64 doubles + 64 ints, 256-aligned

// Prepared operands (views): xj, njl over all j-tiles, xi, ni over all rows.
struct I8Prep {
    const double *xj, *xi, *njl, *ni;
    int64_t n, n_pad;
    int d, dq;
    double s2;
};

I8Shape i8_shape(int64_t n, int64_t n_pad, int kc);
size_t i8_vb_bytes(const I8Shape& h);
size_t i8_vl_bytes(const I8Shape& h);
size_t i8_part_bytes(const I8Shape& h, int64_t n, int kc);
// xj, xi (n_pad x round_up(d, 4) doubles), ni (n_pad), njl (16 n_pad) from X,
// with device arrays inv_l (1 / l_r) and mean (column means of X).
void i8_prepare_into(hipStream_t s, const double* X, int64_t n, int d, const double* inv_l,
                     const double* mean, double* xj, double* xi, double* ni, double* njl);
// Fails unless the buffers (bytes) cover every index the kernels form.
void i8_check_prep(const I8Prep& P, size_t xj, size_t xi, size_t ni, size_t njl);
// One column group: Y = (K + shift I) V for columns [0, kc) of V / Y (leading
// dimensions ldv, ldy).  ctx only times the product launches (NULL: untimed).
void i8_run_group(pkm_ctx* ctx, hipStream_t s, const I8Prep& P, const I8Shape& h,
                  const I8Work& w, int kc, const double* V, int ldv, double* Y, int ldy,
                  double shift);

}  // namespace pkm
