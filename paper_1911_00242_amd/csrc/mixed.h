// Mixed-precision (split-BF16) operands and launchers (internal to libccsdk).
#pragma once
#include "common.h"

namespace ck {

// Grouped complex GEMM on split-BF16 operands; same offset tables as GemmOps.  A and B
// hold four bf16 planes (re_hi, re_lo, im_hi, im_lo) at plane strides a_plane, b_plane
// (elements); C is complex128.  fast = 1 when every aligned group of 8 k indices is
// contiguous and 16-byte aligned in both operands (then loads move 8 k at once).
struct SplitOps {
    const uint16_t *A, *B;
    const uint16_t *zeros;  // >= 16 bytes of zeros: the load address of out-of-range chunks
    int64_t a_plane, b_plane;
    cd *C;
    const int64_t *a_row, *a_k, *b_col, *b_k, *c_row, *c_col;
    int G, M, N, K;
    double alpha, beta;
    int fast;
};

void gemm_split(const SplitOps &op, hipStream_t s);
// dst planes of n elements each (plane stride `plane`) from complex128 src
void launch_split(int64_t n, const cd *src, uint16_t *dst, int64_t plane, hipStream_t st);
// split planes of the per-block (o^2 x v^2) -> (v^2 x o^2) transpose of src
void launch_split_transpose(const Dims &d, const cd *src, uint16_t *dst, int64_t plane, hipStream_t st);
// T1-dressed <ab||ef> written as split planes
void launch_vvvv_dress_split(const SysDev &s, const cd *t1, uint16_t *Vt, int64_t plane, hipStream_t st);

}  // namespace ck
