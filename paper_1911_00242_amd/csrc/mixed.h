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
// Both parts of a complex value at once with the packed hardware conversion
// (v_cvt_pk_bf16_f32, round to nearest even): the same bits as split2 on each part.
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
__device__ inline void split2c(cd x, uint16_t &rh, uint16_t &rl, uint16_t &ih, uint16_t &il) {
    const uint32_t hi = __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2_t{(float)x.x, (float)x.y}, bf16x2_t));
    const double hr = (double)__builtin_bit_cast(float, hi << 16), hm = (double)__builtin_bit_cast(float, hi & 0xffff0000u);
    const uint32_t lo =
        __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2_t{(float)(x.x - hr), (float)(x.y - hm)}, bf16x2_t));
    rh = (uint16_t)hi;
    ih = (uint16_t)(hi >> 16);
    rl = (uint16_t)lo;
    il = (uint16_t)(lo >> 16);
}

// eight consecutive elements e0 .. e0+7 (e0 a multiple of 8) as one 64-byte chunk
__device__ inline void put_chunk(uint16_t *dst, int64_t e0, const cd (&x)[8]) {
    uint16_t h[4][8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        split2c(x[j], h[0][j], h[1][j], h[2][j], h[3][j]);
    }
    uint4 *o = (uint4 *)(dst + split_index(e0, 0));
#pragma unroll
    for (int p = 0; p < 4; ++p)
        o[p] = make_uint4(h[p][0] | (uint32_t)h[p][1] << 16, h[p][2] | (uint32_t)h[p][3] << 16,
                          h[p][4] | (uint32_t)h[p][5] << 16, h[p][6] | (uint32_t)h[p][7] << 16);
}

// One element, or eight consecutive ones, in the storage of an operand family: split
// storage (c64 false) or complex64 storage (c64 true: element e at float2 index e).
__device__ inline void put_elem(uint16_t *dst, int64_t e, cd v, bool c64) {
    if (c64) {
        reinterpret_cast<cf *>(dst)[e] = make_float2((float)v.x, (float)v.y);
        return;
    }
    uint16_t h0, h1, h2, h3;
    split2c(v, h0, h1, h2, h3);
    dst[split_index(e, 0)] = h0;
    dst[split_index(e, 1)] = h1;
    dst[split_index(e, 2)] = h2;
    dst[split_index(e, 3)] = h3;
}
__device__ inline void put_chunk(uint16_t *dst, int64_t e0, const cd (&x)[8], bool c64) {
    if (!c64) {
        put_chunk(dst, e0, x);
        return;
    }
    float4 *o = reinterpret_cast<float4 *>(reinterpret_cast<cf *>(dst) + e0);
#pragma unroll
    for (int q = 0; q < 4; ++q)
        o[q] = make_float4((float)x[2 * q].x, (float)x[2 * q].y, (float)x[2 * q + 1].x, (float)x[2 * q + 1].y);
}

// Grouped complex GEMM on split-BF16 operands; same offset tables as GemmOps (element
// offsets into the unsplit operand, mapped through split_index).  C is complex128.
// fast = 1 when every aligned group of 8 k indices is contiguous and starts at a multiple
// of 8 in both operands (then loads move 8 k of one plane at once).  A column with
// c_col < 0 is padding and is not written.  With Cs set, the result alpha*AB + beta*C is
// written in split storage to Cs at cs_row + cs_col (cs_row/cs_col = NULL: the C offsets)
// and C is only read.
struct SplitOps {
    const uint16_t *A, *B;
    const uint16_t *zeros;  // >= 16 bytes of zeros: the load address of out-of-range chunks
    cd *C;
    uint16_t *Cs;
    const int64_t *a_row, *a_k, *b_col, *b_k, *c_row, *c_col;
    const int64_t *cs_row, *cs_col;
    int G, M, N, K;
    double alpha, beta;
    int fast;
    // entries per group of the k tables (a_k[g * kld + k]); 0: K.  A product over a range of
    // k is then a_k, b_k offset to the range's first k with K its length.
    int64_t kld = 0;
};

void gemm_split(const SplitOps &op, hipStream_t s);

// Arithmetic forms of a mixed-precision product.  PRESPLIT2 runs on split storage (the
// layout above); the other three on complex64 storage (interleaved float2, element e at
// float2 index e; an operand of n elements takes round_up(n, 8) of them, the same bytes
// as its split storage), splitting in registers.
enum Arith { ARITH_PRESPLIT2 = 0, ARITH_SPLIT2 = 1, ARITH_SPLIT3 = 2, ARITH_FP32 = 3, ARITH_COUNT = 4 };
inline bool arith_c64(int a) { return a != ARITH_PRESPLIT2; }
// the product on complex64 operands (A, B, Cs of op read / written as complex64)
void gemm_c64(const SplitOps &op, int arith, hipStream_t s);
// complex64 storage of n complex128 elements (round to nearest; padding zeroed)
void launch_to_c64(int64_t n, const cd *src, cf *dst, hipStream_t st);
// split storage of n complex128 elements (pad of the last chunk zeroed)
void launch_split(int64_t n, const cd *src, uint16_t *dst, hipStream_t st);
// an operand in the storage of its family
inline void launch_operand(int64_t n, const cd *src, uint16_t *dst, bool c64, hipStream_t st) {
    if (c64) launch_to_c64(n, src, reinterpret_cast<cf *>(dst), st);
    else launch_split(n, src, dst, st);
}

}  // namespace ck
