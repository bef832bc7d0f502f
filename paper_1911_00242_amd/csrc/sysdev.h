// The system view of the side kernels (everything but the grouped products): mesh and
// sizes, the device arrays of one system, and momentum and amplitude helpers.
#pragma once
#include "common.h"

namespace ck {

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

// Device views of one system's arrays.
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
    // Mixed-precision path only (null otherwise): the integral classes in complex64, the
    // only copies it keeps (the six complex128 classes above are then null).  They enter
    // the residual scaled by amplitudes, or in sums that are rounded to split bf16 before
    // their products (W_mnij, W_mbej and the dressed <ab||ef>), or (oovv) as the driver
    // term and in the energy, where their rounding errors average out.  vvvv_c holds only
    // the blocks (ka, kb, ke) with ka <= kb and ke <= kf, which contain every pair that is
    // canonical in both (a, b) and (e, f): vblk[block] is a block's place among them (-1:
    // not kept).
    const cf *ovvv_c, *ovvvT_c, *ovvoT_c, *oovvT_c, *oovv_c;
    const cf *oooo_c, *ooov_c, *vvvv_c;
    const int32_t *vblk;
};

// The copy of a class a kernel instantiated for element type IT reads (IT = cf: the
// mixed-precision path).
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
template <class IT> __device__ inline const IT *oooo_of(const SysDev &s);
template <> __device__ inline const cd *oooo_of<cd>(const SysDev &s) { return s.oooo; }
template <> __device__ inline const cf *oooo_of<cf>(const SysDev &s) { return s.oooo_c; }
template <class IT> __device__ inline const IT *ooov_of(const SysDev &s);
template <> __device__ inline const cd *ooov_of<cd>(const SysDev &s) { return s.ooov; }
template <> __device__ inline const cf *ooov_of<cf>(const SysDev &s) { return s.ooov_c; }

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

}  // namespace ck
