// Mixed-precision (split-BF16) operands and launchers (internal to libccsdk).
#pragma once
#include "common.h"

namespace ck {

// Split-BF16 storage: every complex element x becomes four bf16 values (re_hi, re_lo,
// im_hi, im_lo), hi = bf16(x), lo = bf16(x - hi).  They are stored chunk interleaved:
// elements 8c .. 8c+7 of an operand occupy 64 contiguous bytes, plane p at bytes
// 16p .. 16p+15, so the 16-byte loads of the GEMM read whole 128-byte lines for two
// consecutive chunks.  An operand of n elements takes 4 * round_up(n, 8) bf16 values.
__host__ __device__ inline int64_t split_index(int64_t e, int p) { return ((e >> 3) << 5) + (p << 3) + (e & 7); }

// bf16 rounding to nearest even (NaN stays NaN) and the split pair hi = bf16(x),
// lo = bf16(x - hi)
__host__ __device__ inline uint16_t bf16_rne(float f) {
    uint32_t u = __builtin_bit_cast(uint32_t, f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__host__ __device__ inline float bf16_to_f(uint16_t h) { return __builtin_bit_cast(float, (uint32_t)h << 16); }
__host__ __device__ inline void split2(double x, uint16_t &hi, uint16_t &lo) {
    hi = bf16_rne((float)x);
    lo = bf16_rne((float)(x - (double)bf16_to_f(hi)));
}

// Grouped complex GEMM on split-BF16 operands; same offset tables as GemmOps (element
// offsets into the unsplit operand, mapped through split_index).  C is complex128.
// fast = 1 when every aligned group of 8 k indices is contiguous and starts at a multiple
// of 8 in both operands (then loads move 8 k of one plane at once).  With Cs set, the
// result alpha*AB + beta*C is written in split storage to Cs (same element offsets) and C
// is only read.
struct SplitOps {
    const uint16_t *A, *B;
    const uint16_t *zeros;  // >= 16 bytes of zeros: the load address of out-of-range chunks
    cd *C;
    uint16_t *Cs;
    const int64_t *a_row, *a_k, *b_col, *b_k, *c_row, *c_col;
    int G, M, N, K;
    double alpha, beta;
    int fast;
};

void gemm_split(const SplitOps &op, hipStream_t s);
// split storage of n complex128 elements (pad of the last chunk zeroed)
void launch_split(int64_t n, const cd *src, uint16_t *dst, hipStream_t st);
// split storage of the per-block (o^2 x v^2) -> (v^2 x o^2) transpose of src
void launch_split_transpose(const Dims &d, const cd *src, uint16_t *dst, hipStream_t st);
// tau from (t1, t2) straight to split storage: tau, its per-block transpose, and t2 itself;
// needs n_occ^2 and n_vir^2 to be multiples of 8 (tau_split_ok)
bool tau_split_ok(const Dims &d);
void launch_tau_split(const Dims &d, const int32_t *kc, const cd *t1, const cd *t2, uint16_t *tau_s,
                      uint16_t *tauT_s, uint16_t *t2_s, hipStream_t st);
// T1-dressed <ab||ef> written in split storage
void launch_vvvv_dress_split(const SysDev &s, const cd *t1, uint16_t *Vt, hipStream_t st);

}  // namespace ck
