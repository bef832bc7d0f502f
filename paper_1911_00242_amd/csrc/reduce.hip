// FP64 reductions, the plain amplitude update and the DIIS step on the device, plus the
// device twin of the synthetic input recipe.
//
// Reductions are deterministic: a fixed grid of RED_BLOCKS workgroups, each summing a fixed
// strided subset in a fixed order, a fixed LDS tree, and a single-block final pass.
// The update is the paper's successive substitution t <- t + D^-1 R (Sec. 4.4, with
// D_i^a = f_ii - f_aa and D_ij^ab = f_ii + f_jj - f_aa - f_bb).
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

template <int W>
__device__ inline void block_sum(double (&v)[W], double (*sh)[256]) {
    const int t = threadIdx.x;
#pragma unroll
    for (int w = 0; w < W; ++w) sh[w][t] = v[w];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (t < s)
#pragma unroll
            for (int w = 0; w < W; ++w) sh[w][t] += sh[w][t + s];
        __syncthreads();
    }
#pragma unroll
    for (int w = 0; w < W; ++w) v[w] = sh[w][0];
}

// sum of W-wide partial rows: out[w] = sum_b partials[w*nb + b]
template <int W>
__global__ void k_final_sum(const double *partials, int nb, double *out) {
    __shared__ double sh[W][256];
    double v[W];
#pragma unroll
    for (int w = 0; w < W; ++w) {
        double a = 0.0;
        for (int b = threadIdx.x; b < nb; b += 256) a += partials[(int64_t)w * nb + b];
        v[w] = a;
    }
    block_sum<W>(v, sh);
    if (threadIdx.x == 0)
#pragma unroll
        for (int w = 0; w < W; ++w) out[w] = v[w];
}

__global__ void k_norm2(int64_t n1, const cd *r1, int64_t n2, const cd *r2, double *partials) {
    __shared__ double sh[1][256];
    double v[1] = {0.0};
    GRID_STRIDE(i, n1 + n2) {
        cd x = i < n1 ? r1[i] : r2[i - n1];
        v[0] = fma(x.x, x.x, fma(x.y, x.y, v[0]));
    }
    block_sum<1>(v, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = v[0];
}

void launch_norm2(const Dims &d, const cd *r1, const cd *r2, double *partials, double *out, hipStream_t st) {
    hipLaunchKernelGGL(k_norm2, dim3(RED_BLOCKS), dim3(256), 0, st, d.t1(), r1, d.t2(), r2, partials);
    CK_CHECK(hipGetLastError());
    hipLaunchKernelGGL(k_final_sum<1>, dim3(1), dim3(256), 0, st, partials, RED_BLOCKS, out);
    CK_CHECK(hipGetLastError());
}

// E = sum f_ia t_i^a + 1/4 sum <ij||ab> t_ij^ab + 1/2 sum_{ki,kj} <i ki, j kj||a ki, b kj> t_i^a t_j^b
// (<ij||ab> from the complex64 copy on the mixed path, as the energy terms of the
// extrapolation pass)
__global__ void k_energy(SysDev s, const cd *t1, const cd *t2, double *partials) {
    __shared__ double sh[2][256];
    const int N = s.d.N, no = s.d.no, nv = s.d.nv, n = no + nv;
    const int64_t n1 = s.d.t1(), n2 = s.d.t2();
    double v[2] = {0.0, 0.0};
    GRID_STRIDE(idx, n1 + n2) {
        cd p;
        if (idx < n1) {
            int a = (int)(idx % nv), i = (int)((idx / nv) % no), k = (int)(idx / ((int64_t)no * nv));
            p = cmul(s.fock[((int64_t)k * n + i) * n + no + a], t1[idx]);
        } else {
            int64_t e = idx - n1;
            int b = (int)(e % nv), a = (int)((e / nv) % nv);
            int j = (int)((e / ((int64_t)nv * nv)) % no), i = (int)((e / ((int64_t)nv * nv * no)) % no);
            int64_t blk = e / s.d.t2blk();
            int ka = (int)(blk % N), kj = (int)((blk / N) % N), ki = (int)(blk / ((int64_t)N * N));
            cd amp = cscale(t2[e], 0.25);
            if (ka == ki) {
                cd tt = cmul(t1[((int64_t)ki * no + i) * nv + a], t1[((int64_t)kj * no + j) * nv + b]);
                amp = cadd(amp, cscale(tt, 0.5));
            }
            p = cmul(s.oovv_c ? to_cd(s.oovv_c[e]) : s.oovv[e], amp);
        }
        v[0] += p.x;
        v[1] += p.y;
    }
    block_sum<2>(v, sh);
    if (threadIdx.x == 0) {
        partials[blockIdx.x] = v[0];
        partials[RED_BLOCKS + blockIdx.x] = v[1];
    }
}

void launch_energy(const SysDev &s, const cd *t1, const cd *t2, double *partials, double *out, hipStream_t st) {
    hipLaunchKernelGGL(k_energy, dim3(RED_BLOCKS), dim3(256), 0, st, s, t1, t2, partials);
    CK_CHECK(hipGetLastError());
    hipLaunchKernelGGL(k_final_sum<2>, dim3(1), dim3(256), 0, st, partials, RED_BLOCKS, out);
    CK_CHECK(hipGetLastError());
}


template <class R2>
__global__ void k_update(SysDev s, cd *t1, cd *t2, const cd *r1, const R2 *r2, cd *err1, cd *err2, Gate gate) {
    if (!gate.open()) return;
    const int N = s.d.N, no = s.d.no, nv = s.d.nv;
    const int64_t n1 = s.d.t1(), n2 = s.d.t2();
    GRID_STRIDE(idx, n1 + n2) {
        if (idx < n1) {
            int a = (int)(idx % nv), i = (int)((idx / nv) % no), k = (int)(idx / ((int64_t)no * nv));
            double D = s.eo[(int64_t)k * no + i] - s.ev[(int64_t)k * nv + a];
            cd e = make_double2(r1[idx].x / D, r1[idx].y / D);
            t1[idx] = cadd(t1[idx], e);
            if (err1) err1[idx] = e;
        } else {
            int64_t x = idx - n1;
            int b = (int)(x % nv), a = (int)((x / nv) % nv);
            int j = (int)((x / ((int64_t)nv * nv)) % no), i = (int)((x / ((int64_t)nv * nv * no)) % no);
            int64_t blk = x / s.d.t2blk();
            int ka = (int)(blk % N), kj = (int)((blk / N) % N), ki = (int)(blk / ((int64_t)N * N));
            int kb = s.kc[((int64_t)ki * N + kj) * N + ka];
            double D = s.eo[(int64_t)ki * no + i] + s.eo[(int64_t)kj * no + j] - s.ev[(int64_t)ka * nv + a] -
                       s.ev[(int64_t)kb * nv + b];
            const cd rv = to_cd(r2[x]);
            cd e = make_double2(rv.x / D, rv.y / D);
            t2[x] = cadd(t2[x], e);
            if (err2) err2[x] = e;
        }
    }
}

void launch_update(const SysDev &s, cd *t1, cd *t2, const cd *r1, const cd *r2, cd *err1, cd *err2, Gate gate,
                   hipStream_t st) {
    hipLaunchKernelGGL(k_update<cd>, grid_for(s.d.t1() + s.d.t2()), dim3(256), 0, st, s, t1, t2, r1, r2, err1, err2,
                       gate);
    CK_CHECK(hipGetLastError());
}
void launch_update(const SysDev &s, cd *t1, cd *t2, const cd *r1, const cf *r2, cd *err1, cd *err2, Gate gate,
                   hipStream_t st) {
    hipLaunchKernelGGL(k_update<cf>, grid_for(s.d.t1() + s.d.t2()), dim3(256), 0, st, s, t1, t2, r1, r2, err1, err2,
                       gate);
    CK_CHECK(hipGetLastError());
}

// The DIIS step on the device, one workgroup: the overlaps of the new error vector with the
// held ones (sums of the update pass's partials, fixed order) become row and column `slot`
// of B; with two or more vectors held the bordered system
//   [ B 1 ; 1^T 0 ] [ c ; lambda ] = [ 0 ; 1 ]
// is solved by Gaussian elimination with partial pivoting (FP64), otherwise (or when it is
// singular) c is the unit vector of the new slot, i.e. the new amplitudes unchanged.  Then
// the FIFO advances.  Only B's held slots take part, so the FIFO order does not matter.
__global__ __launch_bounds__(256) void k_diis_solve(DiisDev dd, Gate gate, const double *partials, int nparts) {
    if (!gate.open()) return;
    __shared__ double sh[256];
    __shared__ double A[17 * 17], rhs[17];
    const int m = dd.m, slot = dd.state[0], held = min(dd.state[1] + 1, m);
    for (int j = 0; j < held; ++j) {
        double v = 0.0;
        for (int b = threadIdx.x; b < nparts; b += 256) v += partials[(int64_t)j * nparts + b];
        sh[threadIdx.x] = v;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            dd.bnew[j] = sh[0];
            dd.B[slot * m + j] = dd.B[j * m + slot] = sh[0];
        }
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    for (int j = 0; j < m; ++j) dd.coef[j] = 0.0;
    bool ok = held >= 2;
    if (ok) {
        const int n = held + 1;
        for (int i = 0; i < n * n; ++i) A[i] = 0.0;
        for (int i = 0; i < held; ++i)
            for (int j = 0; j < held; ++j) A[i * n + j] = dd.B[i * m + j];
        for (int i = 0; i < held; ++i) A[i * n + held] = A[held * n + i] = 1.0;
        for (int i = 0; i < n; ++i) rhs[i] = 0.0;
        rhs[held] = 1.0;
        for (int col = 0; col < n && ok; ++col) {
            int piv = col;
            for (int i = col + 1; i < n; ++i)
                if (fabs(A[i * n + col]) > fabs(A[piv * n + col])) piv = i;
            if (A[piv * n + col] == 0.0) {
                ok = false;
                break;
            }
            if (piv != col) {
                for (int j = 0; j < n; ++j) {
                    const double x = A[col * n + j];
                    A[col * n + j] = A[piv * n + j];
                    A[piv * n + j] = x;
                }
                const double x = rhs[col];
                rhs[col] = rhs[piv];
                rhs[piv] = x;
            }
            for (int i = col + 1; i < n; ++i) {
                const double f = A[i * n + col] / A[col * n + col];
                for (int j = col; j < n; ++j) A[i * n + j] -= f * A[col * n + j];
                rhs[i] -= f * rhs[col];
            }
        }
        if (ok) {
            for (int i = n - 1; i >= 0; --i) {
                double v = rhs[i];
                for (int j = i + 1; j < n; ++j) v -= A[i * n + j] * rhs[j];
                rhs[i] = v / A[i * n + i];
            }
            for (int j = 0; j < held; ++j) dd.coef[j] = rhs[j];
        }
    }
    if (!ok) dd.coef[slot] = 1.0;
    dd.state[0] = (slot + 1) % m;
    dd.state[1] = held;
}

void launch_diis_solve(const DiisDev &dd, Gate gate, const double *partials, int nparts, hipStream_t st) {
    hipLaunchKernelGGL(k_diis_solve, dim3(1), dim3(256), 0, st, dd, gate, partials, nparts);
    CK_CHECK(hipGetLastError());
}

__global__ void k_diag(Dims d, const cd *fock, double *eo, double *ev) {
    const int n = d.no + d.nv;
    GRID_STRIDE(i, (int64_t)d.N * n) {
        int p = (int)(i % n), k = (int)(i / n);
        double v = fock[((int64_t)k * n + p) * n + p].x;
        if (p < d.no) eo[(int64_t)k * d.no + p] = v;
        else ev[(int64_t)k * d.nv + p - d.no] = v;
    }
}
void launch_diag(const Dims &d, const cd *fock, double *eo, double *ev, hipStream_t st) {
    hipLaunchKernelGGL(k_diag, grid_for((int64_t)d.N * (d.no + d.nv)), dim3(256), 0, st, d, fock, eo, ev);
    CK_CHECK(hipGetLastError());
}

// ------------------------------------------------------------------ synthetic inputs
// Counter-based recipe: stream state s = mix64(mix64(seed) ^ tag); the n-th draw is
// mix64(s + (n+1)*0x9E3779B97F4A7C15) (the splitmix64 sequence of Steele, Lea and Flood);
// u = ((h >> 11) + 0.5) * 2^-53; raw integral g at counter L from draws 2L, 2L+1 by
// Box-Muller; A = ((g_pqrs + g_qpsr) - (g_qprs + g_pqsr))/4; H = (A_pqrs + conj(A_rspq))/2.
// Fock: diagonal, -2 + 1.5u (occupied) or 0.5 + 2.5u (virtual), draw k*n+p of tag 1.
__device__ inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
static inline uint64_t mix64_host(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
__device__ inline double uni(uint64_t st, uint64_t n) {
    return ((double)(mix64(st + (n + 1) * 0x9E3779B97F4A7C15ULL) >> 11) + 0.5) * 0x1.0p-53;
}

__device__ inline int kc_mesh(const Mesh &m, int kp, int kq, int kr) {
    int p2 = kp % m.g2, q2 = kq % m.g2, r2 = kr % m.g2;
    int p1 = (kp / m.g2) % m.g1, q1 = (kq / m.g2) % m.g1, r1 = (kr / m.g2) % m.g1;
    int p0 = kp / (m.g2 * m.g1), q0 = kq / (m.g2 * m.g1), r0 = kr / (m.g2 * m.g1);
    int s0 = ((p0 + q0 - r0) % m.g0 + m.g0) % m.g0;
    int s1 = ((p1 + q1 - r1) % m.g1 + m.g1) % m.g1;
    int s2 = ((p2 + q2 - r2) % m.g2 + m.g2) % m.g2;
    return (s0 * m.g1 + s1) * m.g2 + s2;
}

__device__ inline cd raw_g(const Mesh &m, int n, uint64_t st, double scale, int kp, int kq, int kr, int p,
                           int q, int r, int s) {
    uint64_t L = (((((((uint64_t)kp * m.N + kq) * m.N + kr) * n + p) * n + q) * n + r) * n + s);
    double u1 = uni(st, 2 * L), u2 = uni(st, 2 * L + 1);
    double rad = sqrt(-2.0 * log(u1));
    double ph = 2.0 * M_PI * u2;
    return make_double2(scale * rad * cos(ph), scale * rad * sin(ph));
}

__device__ inline cd anti_A(const Mesh &m, int n, uint64_t st, double scale, int kp, int kq, int kr, int p,
                            int q, int r, int s) {
    int ks = kc_mesh(m, kp, kq, kr);
    cd a = raw_g(m, n, st, scale, kp, kq, kr, p, q, r, s);
    cd b = raw_g(m, n, st, scale, kq, kp, kr, q, p, r, s);
    cd c = raw_g(m, n, st, scale, kp, kq, ks, p, q, s, r);
    cd d = raw_g(m, n, st, scale, kq, kp, ks, q, p, s, r);
    return make_double2(0.25 * ((a.x + d.x) - (b.x + c.x)), 0.25 * ((a.y + d.y) - (b.y + c.y)));
}

// Elements c0 .. c0+len-1 of a class into out[0 .. len-1]; with a block list, element c
// lies in block blist[c / block size] (the class stored on those blocks only).
__global__ void k_synth_eri(Mesh m, int no, int nv, uint64_t st, double scale, int4 dim, int4 off,
                            const int32_t *blist, int64_t c0, int64_t len, cd *out) {
    const int n = no + nv;
    const int64_t blk = (int64_t)dim.x * dim.y * dim.z * dim.w;
    GRID_STRIDE(i, len) {
        const int64_t idx = c0 + i;
        int s = (int)(idx % dim.w), r = (int)((idx / dim.w) % dim.z);
        int q = (int)((idx / ((int64_t)dim.w * dim.z)) % dim.y);
        int p = (int)((idx / ((int64_t)dim.w * dim.z * dim.y)) % dim.x);
        int64_t b = idx / blk;
        if (blist) b = blist[b];
        int kr = (int)(b % m.N), kq = (int)((b / m.N) % m.N), kp = (int)(b / ((int64_t)m.N * m.N));
        int ks = kc_mesh(m, kp, kq, kr);
        int P = p + off.x, Q = q + off.y, R = r + off.z, S = s + off.w;
        cd x = anti_A(m, n, st, scale, kp, kq, kr, P, Q, R, S);
        cd y = anti_A(m, n, st, scale, kr, ks, kp, R, S, P, Q);
        out[i] = make_double2(0.5 * (x.x + y.x), 0.5 * (x.y - y.y));
    }
}

void launch_synth_eri_range(const Mesh &m, int no, int nv, uint64_t seed, double scale, const char *cls,
                            const int32_t *blist, int64_t c0, int64_t len, cd *out, hipStream_t st) {
    int d[4], o[4];
    for (int t = 0; t < 4; ++t) {
        d[t] = cls[t] == 'o' ? no : (cls[t] == 'v' ? nv : no + nv);
        o[t] = cls[t] == 'v' ? no : 0;
    }
    uint64_t state = mix64_host(mix64_host(seed) ^ 2ULL);
    if (len <= 0) return;
    hipLaunchKernelGGL(k_synth_eri, grid_for(len), dim3(256), 0, st, m, no, nv, state, scale,
                       make_int4(d[0], d[1], d[2], d[3]), make_int4(o[0], o[1], o[2], o[3]), blist, c0, len, out);
    CK_CHECK(hipGetLastError());
}

void launch_synth_eri(const Mesh &m, int no, int nv, uint64_t seed, double scale, const char *cls, cd *out,
                      hipStream_t st) {
    int64_t total = (int64_t)m.N * m.N * m.N;
    for (int t = 0; t < 4; ++t) total *= cls[t] == 'o' ? no : (cls[t] == 'v' ? nv : no + nv);
    launch_synth_eri_range(m, no, nv, seed, scale, cls, nullptr, 0, total, out, st);
}

__global__ void k_synth_fock(int N, int no, int nv, uint64_t st, cd *fock) {
    const int n = no + nv;
    GRID_STRIDE(idx, (int64_t)N * n * n) {
        int c = (int)(idx % n), r = (int)((idx / n) % n), k = (int)(idx / ((int64_t)n * n));
        double v = 0.0;
        if (r == c) {
            double u = uni(st, (uint64_t)k * n + r);
            v = r < no ? -2.0 + 1.5 * u : 0.5 + 2.5 * u;
        }
        fock[idx] = make_double2(v, 0.0);
    }
}

void launch_synth_fock(const Mesh &m, int no, int nv, uint64_t seed, cd *fock, hipStream_t st) {
    uint64_t state = mix64_host(mix64_host(seed) ^ 1ULL);
    int64_t total = (int64_t)m.N * (no + nv) * (no + nv);
    hipLaunchKernelGGL(k_synth_fock, grid_for(total), dim3(256), 0, st, m.N, no, nv, state, fock);
    CK_CHECK(hipGetLastError());
}

}  // namespace ck
