// Tile shapes of the FP64 grouped complex product (gemm_f64.hip), chosen per product by the
// autotuner or the caller (all shapes give bitwise the same result), and the chunked form of
// the complex64-operand product (gemm_c64.hip).
#pragma once
#include "common.h"
#include "mixed.h"

namespace ck {

enum F64Tile { F64_TILE_32x32 = 0, F64_TILE_64x64 = 1, F64_TILE_128x64 = 2, F64_TILE_64x128 = 3, F64_TILE_COUNT = 4 };

void gemm_f64_tile(const GemmOps<cd> &op, int tile, hipStream_t s);

// The shape a product starts with: 32 x 32 while 64 x 64 tiles would give fewer than 4096
// workgroups (a few per CU: there the smaller tile keeps more of the chip busy; measured
// up to 3x faster on small products), 64 x 64 otherwise.  The autotuner refines it.
inline int f64_default_tile(int64_t G, int64_t M, int64_t N) {
    return G * ((M + 63) / 64) * ((N + 63) / 64) < 4096 ? F64_TILE_32x32 : F64_TILE_64x64;
}

// The complex64-operand product in arithmetic form arith (ARITH_SPLIT2, ARITH_SPLIT3 or
// ARITH_FP32) with its k range summed in chunks of kchunk (a multiple of 16): FP32
// accumulation within a chunk, FP64 across chunks, in one launch on 64 x 64 tiles (the
// output is read and written once).  Same result, up to the order of the FP64 additions,
// as one launch per chunk.
void gemm_c64_chunked(const SplitOps &op, int arith, int kchunk, hipStream_t s);

}  // namespace ck
