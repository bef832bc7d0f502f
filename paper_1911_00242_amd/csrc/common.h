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

// Momentum mesh: k labels are C-order linear indices into grid[0] x grid[1] x grid[2].
struct Mesh {
    int g0, g1, g2, N;
};

// Sizes of one system.
struct Dims {
    int N, no, nv;
    __host__ __device__ int64_t t1() const { return (int64_t)N * no * nv; }
    __host__ __device__ int64_t t2blk() const { return (int64_t)no * no * nv * nv; }
    __host__ __device__ int64_t t2() const { return (int64_t)N * N * N * t2blk(); }
};

// Device views of one system's arrays (FP64 storage).
struct SysDev {
    Dims d;
    const int32_t *kc;  // [N][N][N] k_s = k_p + k_q - k_r
    const double *eo;   // [N][no]   occupied orbital energies (Fock diagonal)
    const double *ev;   // [N][nv]   virtual orbital energies
    const cd *fock;     // [N][n][n]
    const cd *oooo, *ooov, *oovv, *ovvo, *ovvv, *vvvv;  // [kp][kq][kr][p][q][r][s]
    const cd *ovvoT;  // ovvo with the last two indices swapped: [km][kb][ke][m][b][j][e]
    const cd *ovvvT;  // ovvv with the last two indices swapped: [km][kb][ke][m][b][f][e]
    const cd *oovvT;  // oovv with the last two indices swapped: [km][kn][ke][m][n][f][e]
    // Mixed-precision path only (null otherwise): complex64 copies of the classes the side
    // kernels read (then ovvoT, ovvvT and oovvT above are not kept).  They enter the
    // residual scaled by amplitudes, or next to products formed in split bf16, or (oovv)
    // as the driver term and in the energy, where their rounding errors average out.
    const cf *ovvv_c, *ovvvT_c, *ovvoT_c, *oovvT_c, *oovv_c;
};

// The copy of a class a kernel instantiated for element type IT reads.
template <class IT> __device__ inline const IT *ovvv_of(const SysDev &s);
template <> __device__ inline const cd *ovvv_of<cd>(const SysDev &s) { return s.ovvv; }
template <> __device__ inline const cf *ovvv_of<cf>(const SysDev &s) { return s.ovvv_c; }
template <class IT> __device__ inline const IT *ovvvT_of(const SysDev &s);
template <> __device__ inline const cd *ovvvT_of<cd>(const SysDev &s) { return s.ovvvT; }
template <> __device__ inline const cf *ovvvT_of<cf>(const SysDev &s) { return s.ovvvT_c; }
template <class IT> __device__ inline const IT *ovvoT_of(const SysDev &s);
template <> __device__ inline const cd *ovvoT_of<cd>(const SysDev &s) { return s.ovvoT; }
template <> __device__ inline const cf *ovvoT_of<cf>(const SysDev &s) { return s.ovvoT_c; }
template <class IT> __device__ inline const IT *oovvT_of(const SysDev &s);
template <> __device__ inline const cd *oovvT_of<cd>(const SysDev &s) { return s.oovvT; }
template <> __device__ inline const cf *oovvT_of<cf>(const SysDev &s) { return s.oovvT_c; }
template <class IT> __device__ inline const IT *oovv_of(const SysDev &s);
template <> __device__ inline const cd *oovv_of<cd>(const SysDev &s) { return s.oovv; }
template <> __device__ inline const cf *oovv_of<cf>(const SysDev &s) { return s.oovv_c; }

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

// momentum conservation k_a + k_b - k_c from the device table, and the linear index of a
// momentum block (a, b, c)
__device__ inline int kcv(const int32_t *kc, int N, int a, int b, int c) {
    return kc[((int64_t)a * N + b) * N + c];
}
__device__ inline int64_t blk3(int N, int a, int b, int c) { return ((int64_t)a * N + b) * N + c; }

// tau_{ij}^{ab} = t2 + fac * (d(ka,ki) t_i^a t_j^b - d(kb,ki) t_i^b t_j^a)
__device__ inline cd tau_el(const cd *t1, const cd *t2, int64_t idx, int ki, int kj, int ka, int kb,
                            int i, int j, int a, int b, int no, int nv, double fac) {
    cd v = t2[idx];
    if (ka == ki) {
        cd p = cmul(t1[((int64_t)ki * no + i) * nv + a], t1[((int64_t)kj * no + j) * nv + b]);
        v.x += fac * p.x;
        v.y += fac * p.y;
    }
    if (kb == ki) {
        cd p = cmul(t1[((int64_t)ki * no + i) * nv + b], t1[((int64_t)kj * no + j) * nv + a]);
        v.x -= fac * p.x;
        v.y -= fac * p.y;
    }
    return v;
}

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
