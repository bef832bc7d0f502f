// Elementwise and small-contraction kernels of the CCSD residual (FP64).
//
// Everything here is HBM- or latency-bound: the effective amplitudes tau (end of Sec. 2),
// the F intermediates (eqs. ori_F_oo, ori_F_vv, ori_F_ov), the single-amplitude parts of
// the W intermediates, the T1-dressed particle-particle integrals, the ring seed
// -t_i^e t_m^a <mb||ej>, the assembly of every T2 term that is not one of the five big
// products, and the T1 residual (eq. ori_EqSingle).  The big products are done by the
// grouped GEMM; this file prepares their operands and collects their results.
//
// Index conventions (all arrays complex128, k_b or k_s fixed by conservation):
//   t1[k][i][a], t2/r2/tau[ki][kj][ka][i][j][a][b], tauT[ki][kj][ka][a][b][i][j]
//   class blocks [kp][kq][kr][p][q][r][s]
//   WT[ki][kj][km][i][j][m][n]  = hole-hole intermediate W_{m n i j} (k_n fixed)
//   WR[q][kj][km][j][b][m][e]   = ring intermediate W_{m b e j}, k_b = k_j - q, k_e = k_m - q
//   X [q][ki][kj][i][a][j][b]   = ring product, k_a = k_i + q, k_b = k_j - q
#include "common.h"
#include "terms.h"

namespace ck {

#define GRID_STRIDE(i, total) \
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (total); i += (int64_t)gridDim.x * blockDim.x)

static inline dim3 grid_for(int64_t total) {
    int64_t b = (total + 255) / 256;
    if (b > 1 << 20) b = 1 << 20;
    if (b < 1) b = 1;
    return dim3((unsigned)b);
}

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

// ------------------------------------------------------------------ tau and its transpose
__global__ void k_tau(Dims d, const int32_t *kc, const cd *t1, const cd *t2, cd *tau) {
    const int N = d.N, no = d.no, nv = d.nv;
    GRID_STRIDE(idx, d.t2()) {
        int b = (int)(idx % nv);
        int a = (int)((idx / nv) % nv);
        int j = (int)((idx / ((int64_t)nv * nv)) % no);
        int i = (int)((idx / ((int64_t)nv * nv * no)) % no);
        int64_t blk = idx / d.t2blk();
        int ka = (int)(blk % N), kj = (int)((blk / N) % N), ki = (int)(blk / ((int64_t)N * N));
        int kb = kcv(kc, N, ki, kj, ka);
        tau[idx] = tau_el(t1, t2, idx, ki, kj, ka, kb, i, j, a, b, no, nv, 1.0);
    }
}

// per momentum block: (o^2 x v^2) -> (v^2 x o^2), through a 32x32 LDS tile
__global__ void k_block_transpose(Dims d, const cd *src, cd *dst) {
    __shared__ cd tile[32][33];
    const int R = d.no * d.no, C = d.nv * d.nv;
    const int tr = (R + 31) / 32, tc = (C + 31) / 32;
    int64_t blk = blockIdx.x / (tr * tc);
    int t = (int)(blockIdx.x % (tr * tc));
    int r0 = (t / tc) * 32, c0 = (t % tc) * 32;
    const cd *s = src + blk * d.t2blk();
    cd *o = dst + blk * d.t2blk();
    int tx = threadIdx.x % 32, ty = threadIdx.x / 32;  // 256 threads: 32 x 8
    for (int y = ty; y < 32; y += 8) {
        int r = r0 + y, c = c0 + tx;
        if (r < R && c < C) tile[y][tx] = s[(int64_t)r * C + c];
    }
    __syncthreads();
    for (int y = ty; y < 32; y += 8) {
        int c = c0 + y, r = r0 + tx;
        if (r < R && c < C) o[(int64_t)c * R + r] = tile[tx][y];
    }
}

// ------------------------------------------------------------------ F intermediates
// Fov[k](m,e) = f_me + sum_{kn,n,f} t_n^f <m k, n kn || e k, f kn>
__global__ void k_fov(SysDev s, const cd *t1, cd *Fov) {
    const int N = s.d.N, no = s.d.no, nv = s.d.nv, n = no + nv;
    GRID_STRIDE(idx, (int64_t)N * no * nv) {
        int e = (int)(idx % nv), m = (int)((idx / nv) % no), k = (int)(idx / ((int64_t)no * nv));
        cd acc = s.fock[((int64_t)k * n + m) * n + no + e];
        for (int kn = 0; kn < N; ++kn) {
            const cd *g = s.oovv + blk3(N, k, kn, k) * s.d.t2blk() + (int64_t)m * no * nv * nv;
            const cd *t = t1 + (int64_t)kn * no * nv;
            for (int nn = 0; nn < no; ++nn)
                for (int f = 0; f < nv; ++f) cfma(acc, t[nn * nv + f], g[((int64_t)nn * nv + e) * nv + f]);
        }
        Fov[idx] = acc;
    }
}

// Partial sums of the tau-tilde terms of F_oo and F_vv over one extra momentum.
//   Poo[k][kn](m,i) = 1/2 sum_{ke,n,e,f} taut[k,kn,ke](i,n,e,f) <m k, n kn || e ke, f kf>
//   Pvv[k][km](a,e) = -1/2 sum_{kn,m,n,f} taut[km,kn,k](m,n,a,f) <m km, n kn || e k, f kf>
__global__ void k_foo_partial(SysDev s, const cd *t1, const cd *t2, cd *Poo) {
    const int N = s.d.N, no = s.d.no, nv = s.d.nv;
    GRID_STRIDE(idx, (int64_t)N * N * no * no) {
        int i = (int)(idx % no), m = (int)((idx / no) % no);
        int kn = (int)((idx / ((int64_t)no * no)) % N), k = (int)(idx / ((int64_t)no * no * N));
        cd acc = make_double2(0.0, 0.0);
        for (int ke = 0; ke < N; ++ke) {
            int kf = kcv(s.kc, N, k, kn, ke);
            int64_t b = blk3(N, k, kn, ke) * s.d.t2blk();
            for (int nn = 0; nn < no; ++nn)
                for (int e = 0; e < nv; ++e)
                    for (int f = 0; f < nv; ++f) {
                        int64_t ti = b + (((int64_t)i * no + nn) * nv + e) * nv + f;
                        cd tt = tau_el(t1, t2, ti, k, kn, ke, kf, i, nn, e, f, no, nv, 0.5);
                        cfma(acc, tt, s.oovv[b + (((int64_t)m * no + nn) * nv + e) * nv + f]);
                    }
        }
        Poo[idx] = cscale(acc, 0.5);
    }
}

__global__ void k_fvv_partial(SysDev s, const cd *t1, const cd *t2, cd *Pvv) {
    const int N = s.d.N, no = s.d.no, nv = s.d.nv;
    GRID_STRIDE(idx, (int64_t)N * N * nv * nv) {
        int e = (int)(idx % nv), a = (int)((idx / nv) % nv);
        int km = (int)((idx / ((int64_t)nv * nv)) % N), k = (int)(idx / ((int64_t)nv * nv * N));
        cd acc = make_double2(0.0, 0.0);
        for (int kn = 0; kn < N; ++kn) {
            int kf = kcv(s.kc, N, km, kn, k);
            int64_t b = blk3(N, km, kn, k) * s.d.t2blk();
            for (int mm = 0; mm < no; ++mm)
                for (int nn = 0; nn < no; ++nn)
                    for (int f = 0; f < nv; ++f) {
                        int64_t ti = b + (((int64_t)mm * no + nn) * nv + a) * nv + f;
                        cd tt = tau_el(t1, t2, ti, km, kn, k, kf, mm, nn, a, f, no, nv, 0.5);
                        cfma(acc, tt, s.oovv[b + (((int64_t)mm * no + nn) * nv + e) * nv + f]);
                    }
        }
        Pvv[idx] = cscale(acc, -0.5);
    }
}

// Foo[k](m,i) = f_mi + 1/2 f_mc t_i^c + sum_{kn} t_n^e <m k,n kn||i k,e kn> + sum_kn Poo
// Fvv[k](a,e) = f_ae - 1/2 f_me t_m^a + sum_{km} t_m^f <a k,m km||e k,f km> + sum_km Pvv
// and the combinations used by the T2 equation:
// Fvt[k](b,f) = Fvv(b,f) - 1/2 t_r^b Fov(r,f),  Fot[k](n,j) = Foo(n,j) + 1/2 t_j^c Fov(n,c)
__global__ void k_foo_fvv(SysDev s, const cd *t1, const cd *Fov, const cd *Poo, const cd *Pvv,
                          cd *Foo, cd *Fvv) {
    const int N = s.d.N, no = s.d.no, nv = s.d.nv, n = no + nv;
    const int64_t noo = (int64_t)N * no * no, nvv = (int64_t)N * nv * nv;
    GRID_STRIDE(idx, noo + nvv) {
        if (idx < noo) {
            int i = (int)(idx % no), m = (int)((idx / no) % no), k = (int)(idx / ((int64_t)no * no));
            const cd *fk = s.fock + (int64_t)k * n * n;
            cd acc = fk[m * n + i];
            cd h = make_double2(0.0, 0.0);
            for (int c = 0; c < nv; ++c) cfma(h, fk[m * n + no + c], t1[((int64_t)k * no + i) * nv + c]);
            acc = cadd(acc, cscale(h, 0.5));
            for (int kn = 0; kn < N; ++kn) {
                const cd *g = s.ooov + blk3(N, k, kn, k) * ((int64_t)no * no * no * nv);
                for (int nn = 0; nn < no; ++nn)
                    for (int e = 0; e < nv; ++e)
                        cfma(acc, t1[((int64_t)kn * no + nn) * nv + e], g[(((int64_t)m * no + nn) * no + i) * nv + e]);
                acc = cadd(acc, Poo[(((int64_t)k * N + kn) * no + m) * no + i]);
            }
            Foo[idx] = acc;
        } else {
            int64_t r = idx - noo;
            int e = (int)(r % nv), a = (int)((r / nv) % nv), k = (int)(r / ((int64_t)nv * nv));
            const cd *fk = s.fock + (int64_t)k * n * n;
            cd acc = fk[(no + a) * n + no + e];
            cd h = make_double2(0.0, 0.0);
            for (int m = 0; m < no; ++m) cfma(h, fk[m * n + no + e], t1[((int64_t)k * no + m) * nv + a]);
            acc = csub(acc, cscale(h, 0.5));
            for (int km = 0; km < N; ++km) {
                // <a k, m km || e k, f km> = -<m km, a k || e k, f km>  (ovvv block [km,k,k])
                const cd *g = s.ovvv + blk3(N, km, k, k) * ((int64_t)no * nv * nv * nv);
                cd u = make_double2(0.0, 0.0);
                for (int m = 0; m < no; ++m)
                    for (int f = 0; f < nv; ++f)
                        cfma(u, t1[((int64_t)km * no + m) * nv + f], g[(((int64_t)m * nv + a) * nv + e) * nv + f]);
                acc = csub(acc, u);
                acc = cadd(acc, Pvv[(((int64_t)k * N + km) * nv + a) * nv + e]);
            }
            Fvv[r] = acc;
        }
    }
}

__global__ void k_ftilde(Dims d, const cd *t1, const cd *Foo, const cd *Fvv, const cd *Fov, cd *Fot, cd *Fvt) {
    const int N = d.N, no = d.no, nv = d.nv;
    const int64_t noo = (int64_t)N * no * no, nvv = (int64_t)N * nv * nv;
    GRID_STRIDE(idx, noo + nvv) {
        if (idx < noo) {
            int j = (int)(idx % no), nn = (int)((idx / no) % no), k = (int)(idx / ((int64_t)no * no));
            cd h = make_double2(0.0, 0.0);
            for (int c = 0; c < nv; ++c)
                cfma(h, t1[((int64_t)k * no + j) * nv + c], Fov[((int64_t)k * no + nn) * nv + c]);
            Fot[idx] = cadd(Foo[idx], cscale(h, 0.5));
        } else {
            int64_t r = idx - noo;
            int f = (int)(r % nv), b = (int)((r / nv) % nv), k = (int)(r / ((int64_t)nv * nv));
            cd h = make_double2(0.0, 0.0);
            for (int rr = 0; rr < no; ++rr)
                cfma(h, t1[((int64_t)k * no + rr) * nv + b], Fov[((int64_t)k * no + rr) * nv + f]);
            Fvt[r] = csub(Fvv[r], cscale(h, 0.5));
        }
    }
}

// ------------------------------------------------------------------ hole-hole intermediate
// WT[ki][kj][km](i,j,m,n) = <mn||ij> + t_j^e <mn||ie> - t_i^e <mn||je>   (tau part by GEMM)
__global__ void k_wmnij_init(SysDev s, const cd *t1, cd *WT) {
    const int N = s.d.N, no = s.d.no, nv = s.d.nv;
    const int64_t o4 = (int64_t)no * no * no * no, o3v = (int64_t)no * no * no * nv;
    GRID_STRIDE(idx, (int64_t)N * N * N * o4) {
        int nn = (int)(idx % no), m = (int)((idx / no) % no);
        int j = (int)((idx / ((int64_t)no * no)) % no), i = (int)((idx / ((int64_t)no * no * no)) % no);
        int64_t blk = idx / o4;
        int km = (int)(blk % N), kj = (int)((blk / N) % N), ki = (int)(blk / ((int64_t)N * N));
        int kn = kcv(s.kc, N, ki, kj, km);
        cd acc = s.oooo[blk3(N, km, kn, ki) * o4 + (((int64_t)m * no + nn) * no + i) * no + j];
        const cd *g1 = s.ooov + blk3(N, km, kn, ki) * o3v + (((int64_t)m * no + nn) * no + i) * nv;
        const cd *g2 = s.ooov + blk3(N, km, kn, kj) * o3v + (((int64_t)m * no + nn) * no + j) * nv;
        for (int e = 0; e < nv; ++e) {
            cfma(acc, t1[((int64_t)kj * no + j) * nv + e], g1[e]);
            cd p = cmul(t1[((int64_t)ki * no + i) * nv + e], g2[e]);
            acc = csub(acc, p);
        }
        WT[idx] = acc;
    }
}

// ------------------------------------------------------------------ T1-dressed <ab||ef>
// Vt[ka][kb][ke](a,b,e,f) = <ab||ef> - P(ab) sum_m t_{m kb}^{b} <a ka, m kb || e f>
//   = <ab||ef> + t_m^b <m kb, a ka||ef> - t_m^a <m ka, b kb||ef>
__global__ void k_vvvv_dress(SysDev s, const cd *t1, cd *Vt) {
    const int N = s.d.N, no = s.d.no, nv = s.d.nv;
    const int64_t v4 = (int64_t)nv * nv * nv * nv, ov3 = (int64_t)no * nv * nv * nv;
    GRID_STRIDE(idx, (int64_t)N * N * N * v4) {
        int f = (int)(idx % nv), e = (int)((idx / nv) % nv);
        int b = (int)((idx / ((int64_t)nv * nv)) % nv), a = (int)((idx / ((int64_t)nv * nv * nv)) % nv);
        int64_t blk = idx / v4;
        int ke = (int)(blk % N), kb = (int)((blk / N) % N), ka = (int)(blk / ((int64_t)N * N));
        cd acc = s.vvvv[idx];
        const cd *g1 = s.ovvv + blk3(N, kb, ka, ke) * ov3 + ((int64_t)a * nv + e) * nv + f;
        const cd *g2 = s.ovvv + blk3(N, ka, kb, ke) * ov3 + ((int64_t)b * nv + e) * nv + f;
        for (int m = 0; m < no; ++m) {
            cfma(acc, t1[((int64_t)kb * no + m) * nv + b], g1[(int64_t)m * nv * nv * nv]);
            acc = csub(acc, cmul(t1[((int64_t)ka * no + m) * nv + a], g2[(int64_t)m * nv * nv * nv]));
        }
        Vt[idx] = acc;
    }
}

// ------------------------------------------------------------------ ring intermediate seed
// Z[km][kb][ke](m,n,e,j) = <m km, n kb || e ke, j kj> + sum_f t_j^f <m km, n kb || e ke, f kj>
__global__ void k_ring_z(SysDev s, const cd *t1, cd *Z) {
    const int N = s.d.N, no = s.d.no, nv = s.d.nv;
    const int64_t o3v = (int64_t)no * no * no * nv;
    GRID_STRIDE(idx, (int64_t)N * N * N * o3v) {
        int j = (int)(idx % no), e = (int)((idx / no) % nv);
        int nn = (int)((idx / ((int64_t)no * nv)) % no), m = (int)((idx / ((int64_t)no * nv * no)) % no);
        int64_t blk = idx / o3v;
        int ke = (int)(blk % N), kb = (int)((blk / N) % N), km = (int)(blk / ((int64_t)N * N));
        int kj = kcv(s.kc, N, km, kb, ke);
        // <mn||ej> = -<mn||je>  (ooov block [km,kb,kj])
        cd acc = s.ooov[blk3(N, km, kb, kj) * o3v + (((int64_t)m * no + nn) * no + j) * nv + e];
        acc = make_double2(-acc.x, -acc.y);
        const cd *g = s.oovv + blk3(N, km, kb, ke) * s.d.t2blk() + (((int64_t)m * no + nn) * nv + e) * nv;
        for (int f = 0; f < nv; ++f) cfma(acc, t1[((int64_t)kj * no + j) * nv + f], g[f]);
        Z[idx] = acc;
    }
}

// WR[q][kj][km](j,b,m,e) = <mb||ej> + t_j^f <mb||ef> - t_n^b Z(m,n,e,j)   (t2 part by GEMM)
__global__ void k_ring_w0(SysDev s, const cd *t1, const cd *Z, cd *WR) {
    const int N = s.d.N, no = s.d.no, nv = s.d.nv;
    const int64_t ov = (int64_t)no * nv, blkq = ov * ov;
    const int64_t o3v = (int64_t)no * no * no * nv, ov3 = (int64_t)no * nv * nv * nv;
    GRID_STRIDE(idx, (int64_t)N * N * N * blkq) {
        int e = (int)(idx % nv), m = (int)((idx / nv) % no);
        int b = (int)((idx / ov) % nv), j = (int)((idx / (ov * nv)) % no);
        int64_t blk = idx / blkq;
        int km = (int)(blk % N), kj = (int)((blk / N) % N), q = (int)(blk / ((int64_t)N * N));
        int kb = kcv(s.kc, N, kj, 0, q), ke = kcv(s.kc, N, km, 0, q);
        int64_t bb = blk3(N, km, kb, ke);
        cd acc = s.ovvo[bb * s.d.t2blk() + (((int64_t)m * nv + b) * nv + e) * no + j];
        const cd *g = s.ovvv + bb * ov3 + (((int64_t)m * nv + b) * nv + e) * nv;
        for (int f = 0; f < nv; ++f) cfma(acc, t1[((int64_t)kj * no + j) * nv + f], g[f]);
        const cd *z = Z + bb * o3v + (int64_t)m * no * nv * no + (int64_t)e * no + j;
        for (int nn = 0; nn < no; ++nn)
            acc = csub(acc, cmul(t1[((int64_t)kb * no + nn) * nv + b], z[(int64_t)nn * nv * no]));
        WR[idx] = acc;
    }
}

// Q[ka][kb][ki](m,b,i,j) = sum_e t_i^e <m ka, b kb || e ki, j kj>
__global__ void k_ring_q(SysDev s, const cd *t1, cd *Q) {
    const int N = s.d.N, no = s.d.no, nv = s.d.nv;
    const int64_t o3v = (int64_t)no * no * no * nv;
    GRID_STRIDE(idx, (int64_t)N * N * N * o3v) {
        int j = (int)(idx % no), i = (int)((idx / no) % no);
        int b = (int)((idx / ((int64_t)no * no)) % nv), m = (int)((idx / ((int64_t)no * no * nv)) % no);
        int64_t blk = idx / o3v;
        int ki = (int)(blk % N);
        const cd *g = s.ovvo + blk * s.d.t2blk() + ((int64_t)m * nv + b) * nv * no + j;
        cd acc = make_double2(0.0, 0.0);
        for (int e = 0; e < nv; ++e) cfma(acc, t1[((int64_t)ki * no + i) * nv + e], g[(int64_t)e * no]);
        Q[idx] = acc;
    }
}

// X[q][ki][kj](i,a,j,b) = -sum_m t_m^a Q[ka,kb,ki](m,b,i,j)   (t2 W part by GEMM, beta = 1)
__global__ void k_ring_xinit(SysDev s, const cd *t1, const cd *Q, cd *X) {
    const int N = s.d.N, no = s.d.no, nv = s.d.nv;
    const int64_t ov = (int64_t)no * nv, blkq = ov * ov, o3v = (int64_t)no * no * no * nv;
    GRID_STRIDE(idx, (int64_t)N * N * N * blkq) {
        int b = (int)(idx % nv), j = (int)((idx / nv) % no);
        int a = (int)((idx / ov) % nv), i = (int)((idx / (ov * nv)) % no);
        int64_t blk = idx / blkq;
        int kj = (int)(blk % N), ki = (int)((blk / N) % N), q = (int)(blk / ((int64_t)N * N));
        int ka = kcv(s.kc, N, ki, q, 0), kb = kcv(s.kc, N, kj, 0, q);
        const cd *qq = Q + blk3(N, ka, kb, ki) * o3v + ((int64_t)b * no + i) * no + j;
        cd acc = make_double2(0.0, 0.0);
        for (int m = 0; m < no; ++m) cfma(acc, t1[((int64_t)ka * no + m) * nv + a], qq[(int64_t)m * nv * no * no]);
        X[idx] = make_double2(-acc.x, -acc.y);
    }
}

// ------------------------------------------------------------------ T2 assembly
// r2 = <ab||ij> + P(ab) t_ij^af Fvt(b,f) - P(ij) t_in^ab Fot(n,j) + P(ij)P(ab) X
//      + P(ij) <ab||cj> t_i^c - P(ab) t_r^a <rb||ij>
// (the two ladders are accumulated afterwards by the grouped GEMM)
__device__ inline int64_t xidx(int N, int no, int nv, const int32_t *kc, int k1, int k2, int k3,
                               int x, int y, int z, int w) {
    // element (x at k1, y at k2, z at k3, w) of the ring product, z the "a" slot
    int q = kcv(kc, N, k3, 0, k1);
    int64_t ov = (int64_t)no * nv;
    return ((((int64_t)q * N + k1) * N + k2) * ov + (int64_t)x * nv + z) * ov + (int64_t)y * nv + w;
}

__global__ void k_assemble_r2(SysDev s, const cd *t1, const cd *t2, const cd *Fot, const cd *Fvt,
                              const cd *X, cd *r2) {
    const int N = s.d.N, no = s.d.no, nv = s.d.nv;
    const int64_t o3v = (int64_t)no * no * no * nv, ov3 = (int64_t)no * nv * nv * nv;
    GRID_STRIDE(idx, s.d.t2()) {
        int b = (int)(idx % nv), a = (int)((idx / nv) % nv);
        int j = (int)((idx / ((int64_t)nv * nv)) % no), i = (int)((idx / ((int64_t)nv * nv * no)) % no);
        int64_t blk = idx / s.d.t2blk();
        int ka = (int)(blk % N), kj = (int)((blk / N) % N), ki = (int)(blk / ((int64_t)N * N));
        int kb = kcv(s.kc, N, ki, kj, ka);
        const int64_t bsz = s.d.t2blk();
        cd acc = cconj(s.oovv[idx]);
        // P(ab) t_ij^{af} Fvt[kb](b,f)
        const cd *ta = t2 + blk * bsz + (((int64_t)i * no + j) * nv + a) * nv;
        const cd *tb = t2 + blk3(N, ki, kj, kb) * bsz + (((int64_t)i * no + j) * nv + b) * nv;
        const cd *fb = Fvt + ((int64_t)kb * nv + b) * nv, *fa = Fvt + ((int64_t)ka * nv + a) * nv;
        for (int f = 0; f < nv; ++f) {
            cfma(acc, ta[f], fb[f]);
            acc = csub(acc, cmul(tb[f], fa[f]));
        }
        // -P(ij) t_{i n}^{ab} Fot[kj](n,j), n at kj
        const cd *ti = t2 + blk * bsz + ((int64_t)i * no * nv + a) * nv + b;
        const cd *tj = t2 + blk3(N, kj, ki, ka) * bsz + ((int64_t)j * no * nv + a) * nv + b;
        for (int n = 0; n < no; ++n) {
            acc = csub(acc, cmul(ti[(int64_t)n * nv * nv], Fot[((int64_t)kj * no + n) * no + j]));
            cfma(acc, tj[(int64_t)n * nv * nv], Fot[((int64_t)ki * no + n) * no + i]);
        }
        // P(ij)P(ab) X
        acc = cadd(acc, X[xidx(N, no, nv, s.kc, ki, kj, ka, i, j, a, b)]);
        acc = csub(acc, X[xidx(N, no, nv, s.kc, kj, ki, ka, j, i, a, b)]);
        acc = csub(acc, X[xidx(N, no, nv, s.kc, ki, kj, kb, i, j, b, a)]);
        acc = cadd(acc, X[xidx(N, no, nv, s.kc, kj, ki, kb, j, i, b, a)]);
        // P(ij) <a b||c j> t_i^c with <ab||cj> = -conj(<j kj, c ki || a ka, b kb>)
        const cd *g1 = s.ovvv + blk3(N, kj, ki, ka) * ov3 + (int64_t)j * nv * nv * nv + (int64_t)a * nv + b;
        const cd *g2 = s.ovvv + blk3(N, ki, kj, ka) * ov3 + (int64_t)i * nv * nv * nv + (int64_t)a * nv + b;
        for (int c = 0; c < nv; ++c) {
            acc = csub(acc, cmul(t1[((int64_t)ki * no + i) * nv + c], cconj(g1[(int64_t)c * nv * nv])));
            cfma(acc, t1[((int64_t)kj * no + j) * nv + c], cconj(g2[(int64_t)c * nv * nv]));
        }
        // -P(ab) t_r^a <r b||i j> with <r ka, b kb||ij> = conj(<i ki, j kj || r ka, b kb>)
        const cd *h1 = s.ooov + blk3(N, ki, kj, ka) * o3v + ((int64_t)i * no + j) * no * nv + b;
        const cd *h2 = s.ooov + blk3(N, ki, kj, kb) * o3v + ((int64_t)i * no + j) * no * nv + a;
        for (int r = 0; r < no; ++r) {
            acc = csub(acc, cmul(t1[((int64_t)ka * no + r) * nv + a], cconj(h1[(int64_t)r * nv])));
            cfma(acc, t1[((int64_t)kb * no + r) * nv + b], cconj(h2[(int64_t)r * nv]));
        }
        r2[idx] = acc;
    }
}

// ------------------------------------------------------------------ T1 residual
// P1[k][kx](i,a): the two t2-integral terms summed over all but one extra momentum
//   +1/2 sum_{ke,n,e,f} t2[k,kx,ke](i,n,e,f) <a k, n kx || e ke, f kf>
//   -1/2 sum_{kn,m,n,f} t2[kx,kn,k](m,n,a,f) <m kx, n kn || i k, f kf>
__global__ void k_r1_partial(SysDev s, const cd *t2, cd *P1) {
    const int N = s.d.N, no = s.d.no, nv = s.d.nv;
    const int64_t o3v = (int64_t)no * no * no * nv, ov3 = (int64_t)no * nv * nv * nv;
    GRID_STRIDE(idx, (int64_t)N * N * no * nv) {
        int a = (int)(idx % nv), i = (int)((idx / nv) % no);
        int kx = (int)((idx / ((int64_t)no * nv)) % N), k = (int)(idx / ((int64_t)no * nv * N));
        cd acc = make_double2(0.0, 0.0);
        for (int ke = 0; ke < N; ++ke) {
            // <a k, n kx||e f> = -<n kx, a k||e f>  (ovvv block [kx,k,ke])
            const cd *t = t2 + blk3(N, k, kx, ke) * s.d.t2blk() + (int64_t)i * no * nv * nv;
            const cd *g = s.ovvv + blk3(N, kx, k, ke) * ov3 + (int64_t)a * nv * nv;
            for (int nn = 0; nn < no; ++nn)
                for (int ef = 0; ef < nv * nv; ++ef)
                    acc = csub(acc, cmul(t[(int64_t)nn * nv * nv + ef], g[(int64_t)nn * nv * nv * nv + ef]));
        }
        for (int kn = 0; kn < N; ++kn) {
            const cd *t = t2 + blk3(N, kx, kn, k) * s.d.t2blk() + (int64_t)a * nv;
            const cd *g = s.ooov + blk3(N, kx, kn, k) * o3v + (int64_t)i * nv;
            for (int mm = 0; mm < no; ++mm)
                for (int nn = 0; nn < no; ++nn)
                    for (int f = 0; f < nv; ++f)
                        acc = csub(acc, cmul(t[((int64_t)mm * no + nn) * nv * nv + f],
                                             g[((int64_t)mm * no + nn) * no * nv + f]));
        }
        P1[idx] = cscale(acc, 0.5);
    }
}

// r1 = conj(f_ia) + t_i^c Fvv(a,c) - t_r^a Foo(r,i) + sum_kn t2[k,kn,k](i,n,a,f) Fov[kn](n,f)
//      + sum_kn t_r^c <a k, r kn||i k, c kn> + sum_kx P1
__global__ void k_r1(SysDev s, const cd *t1, const cd *t2, const cd *Foo, const cd *Fvv, const cd *Fov,
                     const cd *P1, cd *r1) {
    const int N = s.d.N, no = s.d.no, nv = s.d.nv, n = no + nv;
    GRID_STRIDE(idx, (int64_t)N * no * nv) {
        int a = (int)(idx % nv), i = (int)((idx / nv) % no), k = (int)(idx / ((int64_t)no * nv));
        cd acc = cconj(s.fock[((int64_t)k * n + i) * n + no + a]);
        for (int c = 0; c < nv; ++c)
            cfma(acc, t1[((int64_t)k * no + i) * nv + c], Fvv[((int64_t)k * nv + a) * nv + c]);
        for (int r = 0; r < no; ++r)
            acc = csub(acc, cmul(t1[((int64_t)k * no + r) * nv + a], Foo[((int64_t)k * no + r) * no + i]));
        for (int kn = 0; kn < N; ++kn) {
            const cd *t = t2 + blk3(N, k, kn, k) * s.d.t2blk() + (int64_t)i * no * nv * nv + (int64_t)a * nv;
            for (int nn = 0; nn < no; ++nn)
                for (int f = 0; f < nv; ++f)
                    cfma(acc, t[(int64_t)nn * nv * nv + f], Fov[((int64_t)kn * no + nn) * nv + f]);
            // <a k, r kn || i k, c kn> = <r kn, a k || c kn, i k>  (ovvo block [kn,k,kn])
            const cd *g = s.ovvo + blk3(N, kn, k, kn) * s.d.t2blk() + (int64_t)a * nv * no + i;
            for (int r = 0; r < no; ++r)
                for (int c = 0; c < nv; ++c)
                    cfma(acc, t1[((int64_t)kn * no + r) * nv + c], g[(int64_t)r * nv * nv * no + (int64_t)c * no]);
            acc = cadd(acc, P1[(((int64_t)k * N + kn) * no + i) * nv + a]);
        }
        r1[idx] = acc;
    }
}

// ------------------------------------------------------------------ launchers
#define LAUNCH(kern, total, ...)                                                   \
    do {                                                                           \
        hipLaunchKernelGGL(kern, grid_for(total), dim3(256), 0, st, __VA_ARGS__);  \
        CK_CHECK(hipGetLastError());                                               \
    } while (0)

void launch_tau(const SysDev &s, const cd *t1, const cd *t2, cd *tau, cd *tauT, hipStream_t st) {
    LAUNCH(k_tau, s.d.t2(), s.d, s.kc, t1, t2, tau);
    if (!tauT) return;
    int R = s.d.no * s.d.no, C = s.d.nv * s.d.nv;
    dim3 g((unsigned)((int64_t)((R + 31) / 32) * ((C + 31) / 32) * s.d.N * s.d.N * s.d.N));
    hipLaunchKernelGGL(k_block_transpose, g, dim3(256), 0, st, s.d, tau, tauT);
    CK_CHECK(hipGetLastError());
}

void launch_f(const SysDev &s, const cd *t1, const cd *t2, FWork w, hipStream_t st) {
    const int64_t N = s.d.N, no = s.d.no, nv = s.d.nv;
    LAUNCH(k_fov, N * no * nv, s, t1, w.Fov);
    LAUNCH(k_foo_partial, N * N * no * no, s, t1, t2, w.Poo);
    LAUNCH(k_fvv_partial, N * N * nv * nv, s, t1, t2, w.Pvv);
    LAUNCH(k_foo_fvv, N * no * no + N * nv * nv, s, t1, w.Fov, w.Poo, w.Pvv, w.Foo, w.Fvv);
    LAUNCH(k_ftilde, N * no * no + N * nv * nv, s.d, t1, w.Foo, w.Fvv, w.Fov, w.Fot, w.Fvt);
}

void launch_wmnij_init(const SysDev &s, const cd *t1, cd *WT, hipStream_t st) {
    const int64_t N = s.d.N, no = s.d.no;
    LAUNCH(k_wmnij_init, N * N * N * no * no * no * no, s, t1, WT);
}

void launch_vvvv_dress(const SysDev &s, const cd *t1, cd *Vt, hipStream_t st) {
    const int64_t N = s.d.N, nv = s.d.nv;
    LAUNCH(k_vvvv_dress, N * N * N * nv * nv * nv * nv, s, t1, Vt);
}

void launch_ring_init(const SysDev &s, const cd *t1, cd *scratch, cd *WR, cd *X, hipStream_t st) {
    const int64_t N = s.d.N, no = s.d.no, nv = s.d.nv;
    const int64_t n3 = N * N * N;
    LAUNCH(k_ring_z, n3 * no * no * no * nv, s, t1, scratch);
    LAUNCH(k_ring_w0, n3 * no * nv * no * nv, s, t1, scratch, WR);
    LAUNCH(k_ring_q, n3 * no * no * no * nv, s, t1, scratch);
    LAUNCH(k_ring_xinit, n3 * no * nv * no * nv, s, t1, scratch, X);
}

void launch_assemble_r2(const SysDev &s, const cd *t1, const cd *t2, const FWork &w, const cd *X, cd *r2,
                        hipStream_t st) {
    LAUNCH(k_assemble_r2, s.d.t2(), s, t1, t2, w.Fot, w.Fvt, X, r2);
}

void launch_r1(const SysDev &s, const cd *t1, const cd *t2, const FWork &w, cd *P1, cd *r1, hipStream_t st) {
    const int64_t N = s.d.N, no = s.d.no, nv = s.d.nv;
    LAUNCH(k_r1_partial, N * N * no * nv, s, t2, P1);
    LAUNCH(k_r1, N * no * nv, s, t1, t2, w.Foo, w.Fvv, w.Fov, P1, r1);
}

}  // namespace ck
