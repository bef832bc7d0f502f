// Grouped complex product on caller-owned device operands that allocates no memory: for
// callers that cannot call hipMalloc (code under HIP graph capture, tight serving loops,
// harnesses that forbid allocation).
//
// The scratch the product needs beyond its operands (the offset tables of the grouped
// kernels, a zero block that out-of-range loads read, and for the split-BF16 variant the
// split copies of both operands) lives in one fixed device array of this file, `scratch`.
// Its device address is looked up once per device, on the first call made with that device
// current, and kept; kernels receive that address, never the array's host-side name.  Every
// call on a device shares the array: two calls that overlap on one GPU (different streams,
// or threads) race on it and must be ordered by the caller.  Each call rewrites everything
// it reads from the array before reading it, on its own stream, with kernels only (no
// memset or copy nodes), so one call can be captured into a graph and replayed.
#include <mutex>

#include "common.h"
#include "mixed.h"
#include "noalloc.h"

namespace ck {

namespace {

constexpr uint64_t SCRATCH_BYTES = 64ull << 20;  // per device, held until the process ends
constexpr int MAX_DEVICES = 64;

static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

std::mutex g_mu;
unsigned char *g_ptr[MAX_DEVICES] = {};

uint64_t up256(uint64_t x) { return (x + 255) & ~(uint64_t)255; }

// Dense row-major operands A [G][M][K], B [G][N][K], C [G][M][N] as offset tables of the
// grouped kernels (element offsets), and 256 zero bytes at zeros.
__global__ __launch_bounds__(256) void k_dense_tables(int G, int M, int N, int K, int64_t *a_row, int64_t *a_k,
                                                      int64_t *b_col, int64_t *c_row, int64_t *c_col,
                                                      unsigned char *zeros) {
    const int64_t gm = (int64_t)G * M, gn = (int64_t)G * N, gk = (int64_t)G * K;
    const int64_t total = 2 * gm + 2 * gn + gk + 256;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < total; x += (int64_t)gridDim.x * blockDim.x) {
        int64_t y = x;
        if (y < gm) { a_row[y] = y * K; continue; }
        y -= gm;
        if (y < gk) { a_k[y] = y % (K > 0 ? K : 1); continue; }
        y -= gk;
        if (y < gn) { b_col[y] = y * K; continue; }
        y -= gn;
        if (y < gm) { c_row[y] = y * N; continue; }
        y -= gm;
        if (y < gn) { c_col[y] = y % N; continue; }
        y -= gn;
        zeros[y] = 0;
    }
}

}  // namespace

uint64_t noalloc_scratch_limit() { return SCRATCH_BYTES; }

uint64_t noalloc_scratch_needed(int G, int M, int N, int K, int variant) {
    const uint64_t gm = (uint64_t)G * M, gn = (uint64_t)G * N, gk = (uint64_t)G * K;
    uint64_t b = 256;                                   // zero block
    b += up256(8 * (2 * gm + 2 * gn + gk));             // tables
    if (variant == 2) {                                 // split operands, 8 bytes per element
        const uint64_t pa = (gm * K + 63) / 64 * 64, pb = (gn * K + 63) / 64 * 64;
        b += up256(8 * pa) + up256(8 * pb);
    }
    return b;
}

int noalloc_zgemm(int G, int M, int N, int K, const double *A, const double *B, double *C, int variant,
                  hipStream_t st, std::string &err) {
    if (G < 1 || M < 1 || N < 1 || K < 0 || !A || !B || !C) {
        err = "bad product arguments (G, M, N >= 1, K >= 0, non-null device pointers)";
        return -1;
    }
    if (variant != 0 && variant != 2) {
        err = "variant must be 0 (FP64 MFMA) or 2 (split-BF16 MFMA)";
        return -1;
    }
    // element offsets of the kernels are int64 and their grid indices int32
    if ((int64_t)G * M * K > (int64_t)1 << 40 || (int64_t)G * N * K > (int64_t)1 << 40 ||
        (int64_t)G * M * N > (int64_t)1 << 40) {
        err = "product too large";
        return -1;
    }
    const uint64_t need = noalloc_scratch_needed(G, M, N, K, variant);
    if (need > SCRATCH_BYTES) {
        err = "the product needs " + std::to_string(need) + " bytes of scratch; the allocation-free entry point has " +
              std::to_string(SCRATCH_BYTES) + " (use ccsd_k_debug_zgemm, which allocates)";
        return -1;
    }
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess || dev < 0 || dev >= MAX_DEVICES) {
        err = std::string("hipGetDevice: ") + hipGetErrorString(e);
        return -3;
    }
    unsigned char *base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (!g_ptr[dev]) {
            void *p = nullptr;
            e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !p) {
                err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
                return -3;
            }
            g_ptr[dev] = (unsigned char *)p;
        }
        base = g_ptr[dev];
    }
    const int64_t gm = (int64_t)G * M, gn = (int64_t)G * N, gk = (int64_t)G * K;
    unsigned char *zeros = base;
    int64_t *tab = (int64_t *)(base + 256);
    int64_t *a_row = tab, *a_k = a_row + gm, *b_col = a_k + gk, *c_row = b_col + gn, *c_col = c_row + gm;
    unsigned char *split = base + 256 + up256(8 * (uint64_t)(2 * gm + 2 * gn + gk));
    const int64_t total = 2 * gm + 2 * gn + gk + 256;
    const int blocks = (int)std::min<int64_t>((total + 255) / 256, 4096);
    hipLaunchKernelGGL(k_dense_tables, dim3(blocks), dim3(256), 0, st, G, M, N, K, a_row, a_k, b_col, c_row, c_col,
                       zeros);
    e = hipGetLastError();
    if (e != hipSuccess) {
        err = std::string("table kernel: ") + hipGetErrorString(e);
        return -3;
    }
    try {
        if (variant == 0) {
            GemmOps<cd> op{};
            op.A = (const cd *)A; op.B = (const cd *)B; op.C = (cd *)C; op.zeros = (const cd *)zeros;
            op.a_row = a_row; op.a_k = a_k; op.b_col = b_col; op.b_k = a_k; op.c_row = c_row; op.c_col = c_col;
            op.G = G; op.M = M; op.N = N; op.K = K; op.alpha = 1.0; op.beta = 0.0;
            gemm_f64(op, st);
        } else {
            const uint64_t pa = ((uint64_t)gm * K + 63) / 64 * 64;
            uint16_t *sA = (uint16_t *)split, *sB = (uint16_t *)(split + up256(8 * pa));
            launch_split(gm * K, (const cd *)A, sA, st);
            launch_split(gn * K, (const cd *)B, sB, st);
            SplitOps so{};
            so.A = sA; so.B = sB; so.C = (cd *)C; so.Cs = nullptr;
            so.zeros = (const uint16_t *)zeros;
            so.a_row = a_row; so.a_k = a_k; so.b_col = b_col; so.b_k = a_k; so.c_row = c_row; so.c_col = c_col;
            so.cs_row = so.cs_col = nullptr;
            so.G = G; so.M = M; so.N = N; so.K = K; so.alpha = 1.0; so.beta = 0.0;
            so.fast = (K % 8 == 0) ? 1 : 0;
            gemm_split(so, st);
        }
    } catch (const HipError &he) {
        err = he.what;
        return -3;
    }
    return 0;
}

}  // namespace ck
