// Allocation-free grouped complex product (noalloc.hip), internal to libccsdk.
#pragma once
#include <string>

#include "common.h"

namespace ck {

// Bytes of the per-device scratch array, and the bytes one product needs of it.
uint64_t noalloc_scratch_limit();
uint64_t noalloc_scratch_needed(int G, int M, int N, int K, int variant);
// C[g] = A[g] . B[g]^T on device operands (complex128, dense row-major A [G][M][K],
// B [G][N][K], C [G][M][N]), variant 0 FP64 MFMA or 2 split-BF16 MFMA, enqueued on st.
// Returns 0, -1 (invalid or too large; err says why) or -3 (device error).
int noalloc_zgemm(int G, int M, int N, int K, const double *A, const double *B, double *C, int variant,
                  hipStream_t st, std::string &err);

}  // namespace ck
