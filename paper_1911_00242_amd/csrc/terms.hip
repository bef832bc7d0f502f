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
#include "mixed.h"
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

// hi = RNE_bf16(x), lo = RNE_bf16(x - hi): the split-BF16 pair of the mixed path
__device__ inline uint16_t rne_bf16(float f) {
    uint32_t u = __builtin_bit_cast(uint32_t, f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ inline void split_rne2(double x, uint16_t &hi, uint16_t &lo) {
    hi = rne_bf16((float)x);
    lo = rne_bf16((float)(x - (double)__builtin_bit_cast(float, (uint32_t)hi << 16)));
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

// Partial sums of the tau-tilde terms of F_oo and F_vv, one per momentum block:
//   Poo[k][kn][ke](m,i) = 1/2 sum_{n,e,f} taut[k,kn,ke](i,n,e,f) <m k, n kn || e ke, f kf>
//   Pvv[k][km][kn](a,e) = -1/2 sum_{m,n,f} taut[km,kn,k](m,n,a,f) <m km, n kn || e k, f kf>
// (one thread per block and output element; the block's rows are shared by a wave)
__global__ void k_foo_partial(SysDev s, const cd *t1, const cd *t2, cd *Poo) {
    const int N = s.d.N, no = s.d.no, nv = s.d.nv;
    GRID_STRIDE(idx, (int64_t)N * N * N * no * no) {
        int i = (int)(idx % no), m = (int)((idx / no) % no);
        int64_t blk = idx / ((int64_t)no * no);
        int ke = (int)(blk % N), kn = (int)((blk / N) % N), k = (int)(blk / ((int64_t)N * N));
        int kf = kcv(s.kc, N, k, kn, ke);
        int64_t b = blk * s.d.t2blk();
        cd acc = make_double2(0.0, 0.0);
        for (int nn = 0; nn < no; ++nn)
            for (int e = 0; e < nv; ++e)
                for (int f = 0; f < nv; ++f) {
                    int64_t ti = b + (((int64_t)i * no + nn) * nv + e) * nv + f;
                    cd tt = tau_el(t1, t2, ti, k, kn, ke, kf, i, nn, e, f, no, nv, 0.5);
                    cfma(acc, tt, s.oovv[b + (((int64_t)m * no + nn) * nv + e) * nv + f]);
                }
        Poo[idx] = cscale(acc, 0.5);
    }
}

__global__ void k_fvv_partial(SysDev s, const cd *t1, const cd *t2, cd *Pvv) {
    const int N = s.d.N, no = s.d.no, nv = s.d.nv;
    GRID_STRIDE(idx, (int64_t)N * N * N * nv * nv) {
        int e = (int)(idx % nv), a = (int)((idx / nv) % nv);
        int64_t pb = idx / ((int64_t)nv * nv);
        int kn = (int)(pb % N), km = (int)((pb / N) % N), k = (int)(pb / ((int64_t)N * N));
        int kf = kcv(s.kc, N, km, kn, k);
        int64_t b = blk3(N, km, kn, k) * s.d.t2blk();
        cd acc = make_double2(0.0, 0.0);
        for (int mm = 0; mm < no; ++mm)
            for (int nn = 0; nn < no; ++nn)
                for (int f = 0; f < nv; ++f) {
                    int64_t ti = b + (((int64_t)mm * no + nn) * nv + a) * nv + f;
                    cd tt = tau_el(t1, t2, ti, km, kn, k, kf, mm, nn, a, f, no, nv, 0.5);
                    cfma(acc, tt, s.oovv[b + (((int64_t)mm * no + nn) * nv + e) * nv + f]);
                }
        Pvv[idx] = cscale(acc, -0.5);
    }
}

// Both tau-tilde sums of F_oo and F_vv read the same two momentum blocks, tau-tilde[p,q,r]
// and <oo||vv>[p,q,r]; one workgroup per block stages them through LDS one n-slab at a
// time (rows (x, e) padded to n_vir+1) and forms
//   Poo[p][q][r](m,i) = 1/2 sum_{n,e,f} taut(i,n,e,f) <mn||ef>     (k = p, kn = q, ke = r)
//   Pvv[r][p][q](a,e) = -1/2 sum_{m,n,f} taut(m,n,a,f) <mn||ef>    (k = r, km = p, kn = q)
constexpr int FB_SLAB = 2176;  // o * v * (v + 1) complex elements per staged slab (o=8, v=16)
inline bool f_blocks_fit(const Dims &d) {
    return (int64_t)d.no * d.nv * (d.nv + 1) <= FB_SLAB && d.no * d.no <= 1024 && d.nv * d.nv <= 1024;
}

constexpr int FB_NT = 1024;
__global__ __launch_bounds__(FB_NT) void k_f_blocks(SysDev s, const cd *t1, const cd *t2, cd *Poo, cd *Pvv) {
    __shared__ cd Ts[FB_SLAB], Gs[FB_SLAB];
    __shared__ cd red[FB_NT];
    const int N = s.d.N, no = s.d.no, nv = s.d.nv, vv = nv * nv, rs = nv + 1;
    const int tid = threadIdx.x;
    const int64_t blk = blockIdx.x;
    const int r = (int)(blk % N), q = (int)((blk / N) % N), p = (int)(blk / ((int64_t)N * N));
    const int kb = kcv(s.kc, N, p, q, r);
    const int64_t base = blk * s.d.t2blk();
    const int oo = no * no, parts = FB_NT / oo;
    const int u = tid % oo, part = tid / oo;  // Foo output (m,i) = u, ef slice = part
    const int um = u / no, ui = u % no;
    const int ef0 = part < parts ? (int)((int64_t)part * vv / parts) : 0;
    const int ef1 = part < parts ? (int)((int64_t)(part + 1) * vv / parts) : 0;
    const int vparts = FB_NT / vv;  // threads per Fvv output (v^2 <= FB_NT)
    const int vo = tid % vv, vpart = tid / vv;
    const int va = vo / nv, ve = vo % nv;
    const int mf0 = vpart < vparts ? (int)((int64_t)vpart * no * nv / vparts) : 0;
    const int mf1 = vpart < vparts ? (int)((int64_t)(vpart + 1) * no * nv / vparts) : 0;
    cd aoo = make_double2(0.0, 0.0), avv = make_double2(0.0, 0.0);
    for (int n = 0; n < no; ++n) {
#pragma unroll 4
        for (int x = tid; x < no * vv; x += FB_NT) {
            const int row = x / vv, e = (x % vv) / nv, f = x % nv;
            const int64_t gi = base + (((int64_t)row * no + n) * nv + e) * nv + f;
            Ts[(row * nv + e) * rs + f] = tau_el(t1, t2, gi, p, q, r, kb, row, n, e, f, no, nv, 0.5);
            Gs[(row * nv + e) * rs + f] = s.oovv[gi];
        }
        __syncthreads();
        for (int ef = ef0; ef < ef1; ++ef) {
            const int e = ef / nv, f = ef % nv;
            cfma(aoo, Ts[(ui * nv + e) * rs + f], Gs[(um * nv + e) * rs + f]);
        }
        for (int mf = mf0; mf < mf1; ++mf) {
            const int m = mf / nv, f = mf % nv;
            cfma(avv, Ts[(m * nv + va) * rs + f], Gs[(m * nv + ve) * rs + f]);
        }
        __syncthreads();
    }
    red[tid] = aoo;
    __syncthreads();
    if (tid < oo) {
        cd sum = make_double2(0.0, 0.0);
        for (int pp = 0; pp < parts; ++pp) sum = cadd(sum, red[pp * oo + tid]);
        Poo[blk * oo + (int64_t)um * no + ui] = cscale(sum, 0.5);
    }
    __syncthreads();
    red[tid] = avv;
    __syncthreads();
    if (tid < vv) {
        cd sum = make_double2(0.0, 0.0);
        for (int pp = 0; pp < vparts; ++pp) sum = cadd(sum, red[pp * vv + tid]);
        Pvv[(((int64_t)r * N + p) * N + q) * vv + tid] = cscale(sum, -0.5);
    }
}

// The two t2-integral sums of the T1 equation read the same t2 block [p,q,r]; one
// workgroup per block stages t2(:, n, :, :), <n q, a p||ef> and <m p, n q||i r, f> through
// LDS one n-slab at a time and forms
//   P1[p][q][r](i,a) += -1/2 sum_{n,e,f} t2(i,n,e,f) <n q, a p || e r, f>   (k = p)
//   P1[r][p][q](i,a) += -1/2 sum_{m,n,f} t2(m,n,a,f) <m p, n q || i r, f>   (k = r)
// written to two partial arrays that k_r1 adds.
constexpr int RB_T = 2176, RB_G = 4352, RB_H = 1152;
inline bool r1_blocks_fit(const Dims &d) {
    return (int64_t)d.no * d.nv * (d.nv + 1) <= RB_T && (int64_t)d.nv * (d.nv * d.nv + 1) <= RB_G &&
           (int64_t)d.no * d.no * (d.nv + 1) <= RB_H && d.no * d.nv <= 1024;
}

constexpr int RB_NT = 1024;
__global__ __launch_bounds__(RB_NT) void k_r1_blocks(SysDev s, const cd *t2, cd *P1a, cd *P1b) {
    __shared__ cd Ts[RB_T], Gs[RB_G], Hs[RB_H];
    __shared__ cd red[RB_NT];
    const int N = s.d.N, no = s.d.no, nv = s.d.nv, vv = nv * nv, rs = nv + 1, gs = vv + 1;
    const int tid = threadIdx.x;
    const int64_t blk = blockIdx.x;
    const int r = (int)(blk % N), q = (int)((blk / N) % N), p = (int)(blk / ((int64_t)N * N));
    const int64_t tb = blk * s.d.t2blk();
    const int64_t ov3 = (int64_t)no * nv * vv, o3v = (int64_t)no * no * no * nv;
    const int64_t gb = blk3(N, q, p, r) * ov3;  // ovvv block [q,p,r]: (n, a, e, f)
    const int64_t hb = blk * o3v;               // ooov block [p,q,r]: (m, n, i, f)
    const int nout = no * nv;                   // outputs (i, a)
    const int parts = RB_NT / nout;             // threads per output
    const int part = tid / nout, oi = tid % nout;
    const int ii = oi / nv, aa = oi % nv;
    const int ef0 = part < parts ? (int)((int64_t)part * vv / parts) : 0;
    const int ef1 = part < parts ? (int)((int64_t)(part + 1) * vv / parts) : 0;
    const int mf0 = part < parts ? (int)((int64_t)part * no * nv / parts) : 0;
    const int mf1 = part < parts ? (int)((int64_t)(part + 1) * no * nv / parts) : 0;
    cd accA = make_double2(0.0, 0.0), accB = make_double2(0.0, 0.0);
    for (int n = 0; n < no; ++n) {
#pragma unroll 4
        for (int x = tid; x < no * vv; x += RB_NT) {  // t2(x, n, e, f)
            const int row = x / vv, e = (x % vv) / nv, f = x % nv;
            Ts[(row * nv + e) * rs + f] = t2[tb + (((int64_t)row * no + n) * nv + e) * nv + f];
        }
#pragma unroll 4
        for (int x = tid; x < nv * vv; x += RB_NT)  // <n q, a p || e r, f>: (a, ef)
            Gs[(x / vv) * gs + x % vv] = s.ovvv[gb + (int64_t)n * nv * vv + x];
        for (int x = tid; x < no * no * nv; x += RB_NT) {  // <m p, n q || i r, f>: (m, i, f)
            const int m = x / (no * nv), i = (x / nv) % no, f = x % nv;
            Hs[(m * no + i) * rs + f] = s.ooov[hb + (((int64_t)m * no + n) * no + i) * nv + f];
        }
        __syncthreads();
        for (int ef = ef0; ef < ef1; ++ef) cfma(accA, Ts[(ii * nv + ef / nv) * rs + ef % nv], Gs[aa * gs + ef]);
        for (int mf = mf0; mf < mf1; ++mf) {
            const int m = mf / nv, f = mf % nv;
            cfma(accB, Ts[(m * nv + aa) * rs + f], Hs[(m * no + ii) * rs + f]);
        }
        __syncthreads();
    }
    red[tid] = accA;
    __syncthreads();
    if (tid < nout) {
        cd sum = make_double2(0.0, 0.0);
        for (int pp = 0; pp < parts; ++pp) sum = cadd(sum, red[pp * nout + tid]);
        P1a[blk * nout + tid] = cscale(sum, -0.5);
    }
    __syncthreads();
    red[tid] = accB;
    __syncthreads();
    if (tid < nout) {
        cd sum = make_double2(0.0, 0.0);
        for (int pp = 0; pp < parts; ++pp) sum = cadd(sum, red[pp * nout + tid]);
        P1b[(((int64_t)r * N + p) * N + q) * nout + tid] = cscale(sum, -0.5);
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
            }
            for (int kk = 0; kk < N * N; ++kk) acc = cadd(acc, Poo[(((int64_t)k * N * N + kk) * no + m) * no + i]);
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
            }
            for (int kk = 0; kk < N * N; ++kk) acc = cadd(acc, Pvv[(((int64_t)k * N * N + kk) * nv + a) * nv + e]);
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
#pragma unroll 8
        for (int e = 0; e < nv; ++e) {
            cfma(acc, t1[((int64_t)kj * no + j) * nv + e], g1[e]);
            cd p = cmul(t1[((int64_t)ki * no + i) * nv + e], g2[e]);
            acc = csub(acc, p);
        }
        WT[idx] = acc;
    }
}

// ------------------------------------------------------------------ XCD-aware block order
// Workgroup w runs on XCD w % 8; give each XCD a contiguous range of logical blocks so
// that neighbouring blocks, which share operand rows, meet in the same L2.  Launch
// xcd_grid(n) workgroups; a workgroup whose logical index is >= n exits.
static inline dim3 xcd_grid(int64_t n) { return dim3((unsigned)(((n + 7) / 8) * 8)); }
__device__ inline int64_t xcd_block(int64_t n) {
    const int64_t per = (n + 7) / 8;
    return (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
}

// ------------------------------------------------------------------ T1-dressed <ab||ef>
// Vt[ka][kb][ke](a,b,e,f) = <ab||ef> - P(ab) sum_m t_{m kb}^{b} <a ka, m kb || e f>
//   = <ab||ef> + t_m^b <m kb, a ka||ef> - t_m^a <m ka, b kb||ef>
// One workgroup per (ka, kb, ke, a), XCD-contiguous order.  The <m kb, a ka||ef> rows of
// its a (o x v^2, reused for every b) and t_{m kb}^b, t_{m ka}^a are staged in LDS, so an
// element costs one <ab||ef> and o <m ka, b kb||ef> global reads; neighbouring a share the
// latter block in L2.
constexpr int DR_G1 = 2048, DR_T1 = 512;
__host__ __device__ inline bool dress_fits(const Dims &d) {
    return (int64_t)d.no * d.nv * d.nv <= DR_G1 && d.no * d.nv <= DR_T1;
}

template <bool SPLIT>
__device__ inline void dress_body(const SysDev &s, const cd *t1, cd *Vt, uint16_t *Vs) {
    __shared__ cd G1[DR_G1];
    __shared__ cd TB[DR_T1];
    __shared__ cd TA[64];
    const int N = s.d.N, no = s.d.no, nv = s.d.nv, vv = nv * nv;
    const int64_t v3 = (int64_t)vv * nv, v4 = v3 * nv, ov3 = (int64_t)no * v3;
    const int64_t nblk = (int64_t)N * N * N * nv;
    const int64_t L = xcd_block(nblk);
    if (L >= nblk) return;
    const int a = (int)(L % nv);
    const int64_t blk = L / nv;
    const int ke = (int)(blk % N), kb = (int)((blk / N) % N), ka = (int)(blk / ((int64_t)N * N));
    const bool lds = dress_fits(s.d);
    const cd *g1b = s.ovvv + blk3(N, kb, ka, ke) * ov3 + (int64_t)a * vv;
    const cd *g2b = s.ovvv + blk3(N, ka, kb, ke) * ov3;
    if (lds) {
        for (int x = threadIdx.x; x < no * vv; x += blockDim.x) G1[x] = g1b[(int64_t)(x / vv) * v3 + x % vv];
        for (int x = threadIdx.x; x < no * nv; x += blockDim.x) TB[x] = t1[(int64_t)kb * no * nv + x];
        for (int x = threadIdx.x; x < no; x += blockDim.x) TA[x] = t1[((int64_t)ka * no + x) * nv + a];
        __syncthreads();
    }
    for (int64_t e = threadIdx.x; e < v3; e += blockDim.x) {
        const int ef = (int)(e % vv), b = (int)(e / vv);
        const int64_t idx = blk * v4 + (int64_t)a * v3 + e;
        cd acc = s.vvvv[idx];
#pragma unroll 8
        for (int m = 0; m < no; ++m) {
            const cd g1 = lds ? G1[m * vv + ef] : g1b[(int64_t)m * v3 + ef];
            const cd tb = lds ? TB[m * nv + b] : t1[((int64_t)kb * no + m) * nv + b];
            const cd ta = lds ? TA[m] : t1[((int64_t)ka * no + m) * nv + a];
            cfma(acc, tb, g1);
            acc = csub(acc, cmul(ta, g2b[(int64_t)m * v3 + (int64_t)b * vv + ef]));
        }
        if (SPLIT) {
            uint16_t p0, p1, p2, p3;
            split_rne2(acc.x, p0, p1);
            split_rne2(acc.y, p2, p3);
            Vs[split_index(idx, 0)] = p0;
            Vs[split_index(idx, 1)] = p1;
            Vs[split_index(idx, 2)] = p2;
            Vs[split_index(idx, 3)] = p3;
        } else {
            Vt[idx] = acc;
        }
    }
}

__global__ __launch_bounds__(256) void k_vvvv_dress(SysDev s, const cd *t1, cd *Vt) {
    dress_body<false>(s, t1, Vt, nullptr);
}
__global__ __launch_bounds__(256) void k_vvvv_dress_split(SysDev s, const cd *t1, uint16_t *Vt) {
    dress_body<true>(s, t1, nullptr, Vt);
}

// ------------------------------------------------------------------ ring intermediate seed
// ovvoT[km][kb][ke](m,b,j,e) = <m km, b kb || e ke, j kj>: the static ovvo class with its
// last two indices swapped, made once per set of inputs so that every ring seed below
// reads contiguous runs.
__global__ void k_ovvo_transpose(SysDev s, cd *ovvoT) {
    const int no = s.d.no, nv = s.d.nv;
    GRID_STRIDE(idx, s.d.t2()) {
        int e = (int)(idx % nv), j = (int)((idx / nv) % no);
        int64_t mb = idx / ((int64_t)no * nv);  // (block, m, b)
        ovvoT[idx] = s.ovvo[(mb * nv + e) * no + j];
    }
}

// Last-two-index swaps of the static ovvv and oovv classes, so that the contractions over
// their last index below read along lanes:  ovvvT[..](m,b,f,e) = <mb||ef>,
// oovvT[..](m,n,f,e) = <mn||ef>.
__global__ void k_swap_last2(int64_t nblocks, int v, const cd *src, cd *dst) {
    const int64_t vv = (int64_t)v * v;
    GRID_STRIDE(idx, nblocks * vv) {
        const int64_t r = idx / vv;
        const int e = (int)(idx % v), f = (int)((idx / v) % v);
        dst[idx] = src[r * vv + (int64_t)e * v + f];
    }
}

// Z[km][kb][ke](m,n,j,e) = <m km, n kb || e ke, j kj> + sum_f t_j^f <m km, n kb || e ke, f kj>
__global__ void k_ring_z(SysDev s, const cd *t1, cd *Z) {
    const int N = s.d.N, no = s.d.no, nv = s.d.nv;
    const int64_t o3v = (int64_t)no * no * no * nv;
    GRID_STRIDE(idx, (int64_t)N * N * N * o3v) {
        int e = (int)(idx % nv), j = (int)((idx / nv) % no);
        int nn = (int)((idx / ((int64_t)nv * no)) % no), m = (int)((idx / ((int64_t)nv * no * no)) % no);
        int64_t blk = idx / o3v;
        int ke = (int)(blk % N), kb = (int)((blk / N) % N), km = (int)(blk / ((int64_t)N * N));
        int kj = kcv(s.kc, N, km, kb, ke);
        // <mn||ej> = -<mn||je>  (ooov block [km,kb,kj])
        cd acc = s.ooov[blk3(N, km, kb, kj) * o3v + (((int64_t)m * no + nn) * no + j) * nv + e];
        acc = make_double2(-acc.x, -acc.y);
        const cd *g = s.oovvT + blk * s.d.t2blk() + ((int64_t)m * no + nn) * nv * nv + e;
        #pragma unroll 8
        for (int f = 0; f < nv; ++f) cfma(acc, t1[((int64_t)kj * no + j) * nv + f], g[(int64_t)f * nv]);
        Z[idx] = acc;
    }
}

// WR[q][kj][km](j,b,m,e) = <mb||ej> + t_j^f <mb||ef> - t_n^b Z(m,n,j,e)   (t2 part by GEMM)
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
        cd acc = s.ovvoT[bb * s.d.t2blk() + (((int64_t)m * nv + b) * no + j) * nv + e];
        const cd *g = s.ovvvT + bb * ov3 + ((int64_t)m * nv + b) * nv * nv + e;
        #pragma unroll 8
        for (int f = 0; f < nv; ++f) cfma(acc, t1[((int64_t)kj * no + j) * nv + f], g[(int64_t)f * nv]);
        const cd *z = Z + bb * o3v + (int64_t)m * no * no * nv + (int64_t)j * nv + e;
        #pragma unroll 8
        for (int nn = 0; nn < no; ++nn)
            acc = csub(acc, cmul(t1[((int64_t)kb * no + nn) * nv + b], z[(int64_t)nn * no * nv]));
        WR[idx] = acc;
    }
}

// Q[ka][kb][ki](m,i,j,b) = sum_e t_i^e <m ka, b kb || e ki, j kj> + 1/2 conj(<i ki, j kj || m ka, b kb>)
__global__ void k_ring_q(SysDev s, const cd *t1, cd *Q) {
    const int N = s.d.N, no = s.d.no, nv = s.d.nv;
    const int64_t o3v = (int64_t)no * no * no * nv;
    GRID_STRIDE(idx, (int64_t)N * N * N * o3v) {
        int b = (int)(idx % nv), j = (int)((idx / nv) % no);
        int i = (int)((idx / ((int64_t)nv * no)) % no), m = (int)((idx / ((int64_t)nv * no * no)) % no);
        int64_t blk = idx / o3v;
        int ki = (int)(blk % N), kb = (int)((blk / N) % N), ka = (int)(blk / ((int64_t)N * N));
        int kj = kcv(s.kc, N, ka, kb, ki);
        const cd *g = s.ovvoT + blk * s.d.t2blk() + (((int64_t)m * nv + b) * no + j) * nv;
        cd acc = make_double2(0.0, 0.0);
        #pragma unroll 8
        for (int e = 0; e < nv; ++e) cfma(acc, t1[((int64_t)ki * no + i) * nv + e], g[e]);
        cd h = s.ooov[blk3(N, ki, kj, ka) * o3v + (((int64_t)i * no + j) * no + m) * nv + b];
        acc.x += 0.5 * h.x;
        acc.y -= 0.5 * h.y;
        Q[idx] = acc;
    }
}

// X[q][ki][kj](i,a,j,b), k_a = k_i + q, k_b = k_j - q: everything of the T2 equation that is
// neither the driver nor a ladder, arranged so that one P(ij)P(ab) produces it:
//   - t_i^e t_m^a <mb||ej>                       (ring, the t2 W_mbej part is added by GEMM)
//   - 1/2 t_i^c <ab||cj>,  - 1/2 t_r^a <rb||ij>  (antisymmetric in ab / in ij, so 1/2 under
//                                                 P(ij)P(ab) gives P(ij) / -P(ab) of them)
//   + 1/2 t_ij^af Fvt(b,f), - 1/2 t_in^ab Fot(n,j) (antisymmetric in ij / in ab, likewise)
// This uses the antisymmetry of t2 in (i,j) and (a,b).
__global__ void k_ring_xinit(SysDev s, const cd *t1, const cd *t2, const cd *Q, const cd *Fot, const cd *Fvt,
                             cd *X) {
    const int N = s.d.N, no = s.d.no, nv = s.d.nv;
    const int64_t ov = (int64_t)no * nv, blkq = ov * ov, o3v = (int64_t)no * no * no * nv;
    const int64_t ov3 = (int64_t)no * nv * nv * nv;
    GRID_STRIDE(idx, (int64_t)N * N * N * blkq) {
        int b = (int)(idx % nv), j = (int)((idx / nv) % no);
        int a = (int)((idx / ov) % nv), i = (int)((idx / (ov * nv)) % no);
        int64_t blk = idx / blkq;
        int kj = (int)(blk % N), ki = (int)((blk / N) % N), q = (int)(blk / ((int64_t)N * N));
        int ka = kcv(s.kc, N, ki, q, 0), kb = kcv(s.kc, N, kj, 0, q);
        cd acc = make_double2(0.0, 0.0);
        // -sum_m t_m^a Q(m,i,j,b)
        const cd *qq = Q + blk3(N, ka, kb, ki) * o3v + ((int64_t)i * no + j) * nv + b;
        #pragma unroll 8
        for (int m = 0; m < no; ++m) cfma(acc, t1[((int64_t)ka * no + m) * nv + a], qq[(int64_t)m * no * no * nv]);
        acc = make_double2(-acc.x, -acc.y);
        // -1/2 sum_c t_i^c conj(<j kj, c ki || a ka, b kb>)
        cd y = make_double2(0.0, 0.0);
        const cd *g = s.ovvv + blk3(N, kj, ki, ka) * ov3 + (int64_t)j * nv * nv * nv + (int64_t)a * nv + b;
        #pragma unroll 8
        for (int c = 0; c < nv; ++c) cfma(y, t1[((int64_t)ki * no + i) * nv + c], cconj(g[(int64_t)c * nv * nv]));
        // +1/2 sum_f t_ij^af Fvt[kb](b,f)  - 1/2 sum_n t_in^ab Fot[kj](n,j)
        const int64_t tb = blk3(N, ki, kj, ka) * s.d.t2blk();
        const cd *ta = t2 + tb + (((int64_t)i * no + j) * nv + a) * nv;
        const cd *fb = Fvt + ((int64_t)kb * nv + b) * nv;
        cd w = make_double2(0.0, 0.0);
        #pragma unroll 8
        for (int f = 0; f < nv; ++f) cfma(w, ta[f], fb[f]);
        const cd *tn = t2 + tb + ((int64_t)i * no * nv + a) * nv + b;
        #pragma unroll 8
        for (int n = 0; n < no; ++n) cfma(y, tn[(int64_t)n * nv * nv], Fot[((int64_t)kj * no + n) * no + j]);
        acc.x += 0.5 * (w.x - y.x);
        acc.y += 0.5 * (w.y - y.y);
        X[idx] = acc;
    }
}

// ------------------------------------------------------------------ T2 assembly
// r2 = <ab||ij> + P(ij)P(ab) X   (the two ladders are accumulated afterwards by GEMM).
// One workgroup per (ki,kj,ka,i,j): the two X reads with a and b exchanged go through
// LDS so that every global access is contiguous.  The four terms are added as
// (x1 + x4) - (x2 + x3), which is exactly antisymmetric under i<->j and a<->b.
__device__ inline int64_t xidx(int N, int no, int nv, const int32_t *kc, int k1, int k2, int k3,
                               int x, int y, int z, int w) {
    // element (x at k1, y at k2, z at k3, w) of the ring product, z the "a" slot
    int q = kcv(kc, N, k3, 0, k1);
    int64_t ov = (int64_t)no * nv;
    return ((((int64_t)q * N + k1) * N + k2) * ov + (int64_t)x * nv + z) * ov + (int64_t)y * nv + w;
}

constexpr int ASM_VMAX = 32;

__global__ void k_assemble_r2(SysDev s, const cd *X, cd *r2) {
    __shared__ cd T3[ASM_VMAX * (ASM_VMAX + 1)], T4[ASM_VMAX * (ASM_VMAX + 1)];
    const int N = s.d.N, no = s.d.no, nv = s.d.nv, vv = nv * nv;
    const int64_t nblk = (int64_t)N * N * N * no * no;
    const int64_t L = xcd_block(nblk);
    if (L >= nblk) return;
    const int j = (int)(L % no), i = (int)((L / no) % no);
    const int64_t blk = L / ((int64_t)no * no);
    const int ka = (int)(blk % N), kj = (int)((blk / N) % N), ki = (int)(blk / ((int64_t)N * N));
    const int kb = kcv(s.kc, N, ki, kj, ka);
    const bool lds = nv <= ASM_VMAX;
    if (lds) {
        for (int e = threadIdx.x; e < vv; e += blockDim.x) {
            const int b = e / nv, a = e % nv;  // contiguous in a
            T3[b * (nv + 1) + a] = X[xidx(N, no, nv, s.kc, ki, kj, kb, i, j, b, a)];
            T4[b * (nv + 1) + a] = X[xidx(N, no, nv, s.kc, kj, ki, kb, j, i, b, a)];
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < vv; e += blockDim.x) {
        const int a = e / nv, b = e % nv;
        const int64_t o = blk * s.d.t2blk() + ((int64_t)i * no + j) * vv + e;
        const cd x1 = X[xidx(N, no, nv, s.kc, ki, kj, ka, i, j, a, b)];
        const cd x2 = X[xidx(N, no, nv, s.kc, kj, ki, ka, j, i, a, b)];
        const cd x3 = lds ? T3[b * (nv + 1) + a] : X[xidx(N, no, nv, s.kc, ki, kj, kb, i, j, b, a)];
        const cd x4 = lds ? T4[b * (nv + 1) + a] : X[xidx(N, no, nv, s.kc, kj, ki, kb, j, i, b, a)];
        const cd d = cconj(s.oovv[o]);
        r2[o] = make_double2(d.x + ((x1.x + x4.x) - (x2.x + x3.x)), d.y + ((x1.y + x4.y) - (x2.y + x3.y)));
    }
}

// ------------------------------------------------------------------ T1 residual
// P1[k][kx][ky](i,a): the two t2-integral terms of the T1 equation, one momentum block each
//   +1/2 sum_{n,e,f} t2[k,kx,ky](i,n,e,f) <a k, n kx || e ky, f kf>        (ky = k_e)
//   -1/2 sum_{m,n,f} t2[kx,ky,k](m,n,a,f) <m kx, n ky || i k, f kf>        (kx = k_m, ky = k_n)
__global__ void k_r1_partial(SysDev s, const cd *t2, cd *P1) {
    const int N = s.d.N, no = s.d.no, nv = s.d.nv;
    const int64_t o3v = (int64_t)no * no * no * nv, ov3 = (int64_t)no * nv * nv * nv;
    GRID_STRIDE(idx, (int64_t)N * N * N * no * nv) {
        int a = (int)(idx % nv), i = (int)((idx / nv) % no);
        int64_t pb = idx / ((int64_t)no * nv);
        int ky = (int)(pb % N), kx = (int)((pb / N) % N), k = (int)(pb / ((int64_t)N * N));
        cd acc = make_double2(0.0, 0.0);
        {
            // <a k, n kx||e f> = -<n kx, a k||e f>  (ovvv block [kx,k,ky])
            const cd *t = t2 + blk3(N, k, kx, ky) * s.d.t2blk() + (int64_t)i * no * nv * nv;
            const cd *g = s.ovvv + blk3(N, kx, k, ky) * ov3 + (int64_t)a * nv * nv;
            for (int nn = 0; nn < no; ++nn)
                for (int ef = 0; ef < nv * nv; ++ef)
                    acc = csub(acc, cmul(t[(int64_t)nn * nv * nv + ef], g[(int64_t)nn * nv * nv * nv + ef]));
        }
        {
            const cd *t = t2 + blk3(N, kx, ky, k) * s.d.t2blk() + (int64_t)a * nv;
            const cd *g = s.ooov + blk3(N, kx, ky, k) * o3v + (int64_t)i * nv;
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
                     const cd *P1, int nparts, cd *r1) {
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
        }
        const int64_t np = (int64_t)N * N * N * no * nv;
        for (int pp = 0; pp < nparts; ++pp)
            for (int kk = 0; kk < N * N; ++kk)
                acc = cadd(acc, P1[pp * np + (((int64_t)k * N * N + kk) * no + i) * nv + a]);
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
    if (f_blocks_fit(s.d)) {
        hipLaunchKernelGGL(k_f_blocks, dim3((unsigned)(N * N * N)), dim3(FB_NT), 0, st, s, t1, t2, w.Poo, w.Pvv);
        CK_CHECK(hipGetLastError());
    } else {
        LAUNCH(k_foo_partial, N * N * N * no * no, s, t1, t2, w.Poo);
        LAUNCH(k_fvv_partial, N * N * N * nv * nv, s, t1, t2, w.Pvv);
    }
    LAUNCH(k_foo_fvv, N * no * no + N * nv * nv, s, t1, w.Fov, w.Poo, w.Pvv, w.Foo, w.Fvv);
    LAUNCH(k_ftilde, N * no * no + N * nv * nv, s.d, t1, w.Foo, w.Fvv, w.Fov, w.Fot, w.Fvt);
}

void launch_wmnij_init(const SysDev &s, const cd *t1, cd *WT, hipStream_t st) {
    const int64_t N = s.d.N, no = s.d.no;
    LAUNCH(k_wmnij_init, N * N * N * no * no * no * no, s, t1, WT);
}

void launch_vvvv_dress(const SysDev &s, const cd *t1, cd *Vt, hipStream_t st) {
    const int64_t N = s.d.N, nv = s.d.nv;
    hipLaunchKernelGGL(k_vvvv_dress, xcd_grid(N * N * N * nv), dim3(256), 0, st, s, t1, Vt);
    CK_CHECK(hipGetLastError());
}

void launch_vvvv_dress_split(const SysDev &s, const cd *t1, uint16_t *Vt, hipStream_t st) {
    const int64_t N = s.d.N, nv = s.d.nv;
    hipLaunchKernelGGL(k_vvvv_dress_split, xcd_grid(N * N * N * nv), dim3(256), 0, st, s, t1, Vt);
    CK_CHECK(hipGetLastError());
}

void launch_ovvo_transpose(const SysDev &s, cd *ovvoT, hipStream_t st) {
    LAUNCH(k_ovvo_transpose, s.d.t2(), s, ovvoT);
}

void launch_static_swaps(const SysDev &s, cd *ovvvT, cd *oovvT, hipStream_t st) {
    const int64_t N3 = (int64_t)s.d.N * s.d.N * s.d.N, o = s.d.no, v = s.d.nv;
    LAUNCH(k_swap_last2, N3 * o * v * v * v, N3 * o * v, (int)v, s.ovvv, ovvvT);
    LAUNCH(k_swap_last2, N3 * o * o * v * v, N3 * o * o, (int)v, s.oovv, oovvT);
}

void launch_ring_init(const SysDev &s, const cd *t1, const cd *t2, const FWork &w, cd *scratch, cd *WR, cd *X,
                      hipStream_t st) {
    const int64_t N = s.d.N, no = s.d.no, nv = s.d.nv;
    const int64_t n3 = N * N * N;
    LAUNCH(k_ring_z, n3 * no * no * no * nv, s, t1, scratch);
    LAUNCH(k_ring_w0, n3 * no * nv * no * nv, s, t1, scratch, WR);
    LAUNCH(k_ring_q, n3 * no * no * no * nv, s, t1, scratch);
    LAUNCH(k_ring_xinit, n3 * no * nv * no * nv, s, t1, t2, scratch, w.Fot, w.Fvt, X);
}

void launch_assemble_r2(const SysDev &s, const cd *X, cd *r2, hipStream_t st) {
    const int64_t N = s.d.N, no = s.d.no;
    hipLaunchKernelGGL(k_assemble_r2, xcd_grid(N * N * N * no * no), dim3(256), 0, st, s, X, r2);
    CK_CHECK(hipGetLastError());
}

void launch_r1(const SysDev &s, const cd *t1, const cd *t2, const FWork &w, cd *P1, cd *r1, hipStream_t st) {
    const int64_t N = s.d.N, no = s.d.no, nv = s.d.nv;
    const int64_t np = N * N * N * no * nv;  // P1 holds two partial arrays of np elements
    if (r1_blocks_fit(s.d)) {
        hipLaunchKernelGGL(k_r1_blocks, dim3((unsigned)(N * N * N)), dim3(RB_NT), 0, st, s, t2, P1, P1 + np);
        CK_CHECK(hipGetLastError());
        LAUNCH(k_r1, N * no * nv, s, t1, t2, w.Foo, w.Fvv, w.Fov, P1, 2, r1);
    } else {
        LAUNCH(k_r1_partial, N * N * N * no * nv, s, t2, P1);
        LAUNCH(k_r1, N * no * nv, s, t1, t2, w.Foo, w.Fvv, w.Fov, P1, 1, r1);
    }
}

}  // namespace ck
