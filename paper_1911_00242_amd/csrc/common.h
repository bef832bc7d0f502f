// Internal declarations shared by the HIP translation units of libccsdk.
// Complex numbers are interleaved (re, im): double2 in FP64 storage, float2 in FP32.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#define CK_CHECK(expr)                                                           \
    do {                                                                         \
        hipError_t e_ = (expr);                                                  \
        if (e_ != hipSuccess) throw ck::HipError(e_, #expr, __FILE__, __LINE__); \
    } while (0)

namespace ck {

struct HipError {
    hipError_t code;
    std::string what;
    HipError(hipError_t c, const char *expr, const char *file, int line)
        : code(c),
          what(std::string(hipGetErrorString(c)) + " in " + expr + " at " + file + ":" +
               std::to_string(line)) {}
};

using cd = double2;
using cf = float2;

__host__ __device__ inline cd cmul(cd a, cd b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ inline cd cadd(cd a, cd b) { return make_double2(a.x + b.x, a.y + b.y); }
__host__ __device__ inline cd csub(cd a, cd b) { return make_double2(a.x - b.x, a.y - b.y); }
__host__ __device__ inline cd cscale(cd a, double s) { return make_double2(a.x * s, a.y * s); }
__host__ __device__ inline cd cconj(cd a) { return make_double2(a.x, -a.y); }
// an element of a complex64 copy widened to complex128 (and the identity on complex128)
__host__ __device__ inline cd to_cd(cd v) { return v; }
__host__ __device__ inline cd to_cd(cf v) { return make_double2((double)v.x, (double)v.y); }
// and back: y = x, rounded to complex64 for a complex64 y
__host__ __device__ inline void from_cd(cd x, cd &y) { y = x; }
__host__ __device__ inline void from_cd(cd x, cf &y) { y = make_float2((float)x.x, (float)x.y); }
// a += b * c
__host__ __device__ inline void cfma(cd &a, cd b, cd c) {
    a.x = fma(b.x, c.x, fma(-b.y, c.y, a.x));
    a.y = fma(b.x, c.y, fma(b.y, c.x, a.y));
}

// ---------------------------------------------------------------------------------
// Grouped complex GEMM with gathered operands (all element offsets in complex units):
//   C(g,m,n) = alpha * sum_k A(g,m,k) * B(g,k,n) + beta * C(g,m,n)
//   A(g,m,k) = A[a_row[g*M+m] + a_k[g*K+k]],  B(g,k,n) = B[b_col[g*N+n] + b_k[g*K+k]]
//   C(g,m,n) = C[c_row[g*M+m] + c_col[g*N+n]]
// ---------------------------------------------------------------------------------
template <class T>
struct GemmOps {
    const T *A;
    const T *B;
    T *C;
    const T *zeros;  // >= 16 bytes of zeros: the load address of out-of-range elements
    const int64_t *a_row, *a_k, *b_col, *b_k, *c_row, *c_col;
    int G, M, N, K;
    double alpha, beta;
};

// Tile order of the grouped GEMMs.  Workgroups are dealt to the eight XCDs round robin
// in launch order and each XCD has its own L2, so each XCD is given one contiguous run of
// logical tiles, and each run is walked group_m row tiles at a time: the workgroups
// resident together on an XCD then share a few A row panels and B column panels in its
// L2 instead of each fetching its own pair.  The grid is gemm_tile_grid(...) workgroups
// along x; a workgroup with valid == false has no tile and exits.
struct GemmTile {
    int g, mt, nt;
    bool valid;
};
constexpr int XCDS = 8;
inline dim3 gemm_tile_grid(int tiles_m, int tiles_n, int G) {
    const int64_t t = (int64_t)tiles_m * tiles_n * G;
    return dim3((unsigned)((t + XCDS - 1) / XCDS * XCDS));
}
__device__ inline GemmTile gemm_tile(int tiles_m, int tiles_n, int G, int group_m) {
    const int64_t per_group = (int64_t)tiles_m * tiles_n;
    const int64_t total = per_group * G;
    const int64_t per_xcd = (total + XCDS - 1) / XCDS;
    const int64_t L = (int64_t)(blockIdx.x % XCDS) * per_xcd + blockIdx.x / XCDS;
    GemmTile r;
    r.valid = L < total;
    const int64_t Lc = r.valid ? L : 0;
    r.g = (int)(Lc / per_group);
    const int64_t t = Lc % per_group;
    const int64_t width = (int64_t)group_m * tiles_n;  // tiles in one band of group_m rows
    const int first = (int)(t / width) * group_m;
    const int rows = min(tiles_m - first, group_m);
    const int64_t u = t % width;
    r.mt = first + (int)(u % rows);
    r.nt = (int)(u / rows);
    return r;
}

void gemm_f64(const GemmOps<cd> &op, hipStream_t s);
void gemm_f64_reference(const GemmOps<cd> &op, hipStream_t s);

}  // namespace ck
