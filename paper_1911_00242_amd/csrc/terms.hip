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

// Partial sums of the tau-tilde terms of F_oo and F_vv, one per momentum block:
//   Poo[k][kn][ke](m,i) = 1/2 sum_{n,e,f} taut[k,kn,ke](i,n,e,f) <m k, n kn || e ke, f kf>
//   Pvv[k][km][kn](a,e) = -1/2 sum_{m,n,f} taut[km,kn,k](m,n,a,f) <m km, n kn || e k, f kf>
// (one thread per block and output element; the block's rows are shared by a wave)
template <class IT>
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
                    cfma(acc, tt, to_cd(oovv_of<IT>(s)[b + (((int64_t)m * no + nn) * nv + e) * nv + f]));
                }
        Poo[idx] = cscale(acc, 0.5);
    }
}

template <class IT>
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
                    cfma(acc, tt, to_cd(oovv_of<IT>(s)[b + (((int64_t)mm * no + nn) * nv + e) * nv + f]));
                }
        Pvv[idx] = cscale(acc, -0.5);
    }
}

// Both tau-tilde sums of F_oo and F_vv read the same two momentum blocks, tau-tilde[p,q,r]
// and <oo||vv>[p,q,r]; one workgroup per block stages them through LDS one n-slab at a
// time (rows (x, e) padded to n_vir+1) and forms
//   Poo[p][q][r](m,i) = 1/2 sum_{n,e,f} taut(i,n,e,f) <mn||ef>     (k = p, kn = q, ke = r)
//   Pvv[r][p][q](a,e) = -1/2 sum_{m,n,f} taut(m,n,a,f) <mn||ef>    (k = r, km = p, kn = q)
// When a whole n-slab (o v (v+1) elements) does not fit FB_SLAB, the two sums take
// separate passes: Poo over slabs of every row x and a range of e, Pvv over slabs of a
// range of rows m and every e.  With fr_splits > 1 each pass's list of slabs is cut into
// that many contiguous ranges, one workgroup each (grid splits x N^3), and split sp writes
// its partial sums to slice sp of Poo and Pvv.
constexpr int FB_SLAB = 2176;  // staged complex elements per operand
inline bool f_blocks_fit(const Dims &d) { return d.no <= 32 && d.nv <= 32; }

constexpr int FB_NT = 1024;
template <class IT>  // element type of the <oo||vv> copy read (complex64 on the mixed path)
__global__ __launch_bounds__(FB_NT) void k_f_blocks(SysDev s, const cd *t1, const cd *t2, cd *Poo, cd *Pvv) {
    static_assert(FB_NT <= FB_SLAB, "the reduction reuses the t slab");
    __shared__ cd Ts[FB_SLAB], Gs[FB_SLAB];
    cd *red = Ts;  // after the last slab
    const int N = s.d.N, no = s.d.no, nv = s.d.nv, vv = nv * nv, rs = nv + 1;
    const int tid = threadIdx.x;
    const int64_t n3 = (int64_t)N * N * N;
    const int64_t blk = blockIdx.x % n3;
    const int sp = (int)(blockIdx.x / n3), ns = fr_splits(s.d);
    const int r = (int)(blk % N), q = (int)((blk / N) % N), p = (int)(blk / ((int64_t)N * N));
    const int kb = kcv(s.kc, N, p, q, r);
    const int64_t base = blk * s.d.t2blk();
    const int oo = no * no, parts = FB_NT / oo;
    const int u = tid % oo, part = tid / oo;  // Foo output (m,i) = u, slice = part
    const int um = u / no, ui = u % no;
    // Fvv: a thread per output pair (a, e), (a + ha, e), which share every <mn||ef> read
    const int ha = (nv + 1) / 2, hv = ha * nv;
    const int vparts = FB_NT / hv;  // threads per output pair (ha n_vir <= FB_NT)
    const int vo = tid % hv, vpart = tid / hv;
    const int va = vo / nv, ve = vo % nv;
    const bool two = va + ha < nv;      // the second output exists (odd n_vir)
    const int va2 = two ? va + ha : va;  // (a duplicate read otherwise, discarded)
    // slab of rows x0 .. x0+nx-1 and e0 .. e0+ne-1 of n: element (x, e, f) at
    // ((x - x0) * ne + e - e0) * rs + f
    auto stage = [&](int n, int x0, int nx, int e0, int ne) {
        const int per = ne * nv;
#pragma unroll 4
        for (int x = tid; x < nx * per; x += FB_NT) {
            const int row = x / per, e = (x % per) / nv, f = x % nv;
            const int64_t gi = base + (((int64_t)(x0 + row) * no + n) * nv + e0 + e) * nv + f;
            Ts[(row * ne + e) * rs + f] = tau_el(t1, t2, gi, p, q, r, kb, x0 + row, n, e0 + e, f, no, nv, 0.5);
            Gs[(row * ne + e) * rs + f] = to_cd(oovv_of<IT>(s)[gi]);
        }
    };
    auto slice = [](int pt, int np, int cnt, int &b0, int &b1) {
        b0 = pt < np ? (int)((int64_t)pt * cnt / np) : 0;
        b1 = pt < np ? (int)((int64_t)(pt + 1) * cnt / np) : 0;
    };
    const bool one = (int64_t)no * nv * rs <= FB_SLAB;  // both sums from one slab per n
    const int ec = one ? nv : FB_SLAB / (no * rs), nes = (nv + ec - 1) / ec;
    cd aoo = make_double2(0.0, 0.0), avv = make_double2(0.0, 0.0), avv2 = make_double2(0.0, 0.0);
    // this split's range of the slabs (n, e0), n-major
    const int a0 = sp * no * nes / ns, a1 = (sp + 1) * no * nes / ns;
    for (int it = a0; it < a1; ++it) {
        const int n = it / nes, e0 = (it % nes) * ec;
        const int ne = min(ec, nv - e0);
        stage(n, 0, no, e0, ne);
        __syncthreads();
        int b0, b1;
        slice(part, parts, ne * nv, b0, b1);
        for (int ef = b0; ef < b1; ++ef) {
            const int e = ef / nv, f = ef % nv;
            cfma(aoo, Ts[(ui * ne + e) * rs + f], Gs[(um * ne + e) * rs + f]);
        }
        if (one) {
            slice(vpart, vparts, no * nv, b0, b1);
            for (int mf = b0; mf < b1; ++mf) {
                const int m = mf / nv, f = mf % nv;
                const cd g = Gs[(m * nv + ve) * rs + f];
                cfma(avv, Ts[(m * nv + va) * rs + f], g);
                cfma(avv2, Ts[(m * nv + va2) * rs + f], g);
            }
        }
        __syncthreads();
    }
    if (!one) {
        const int mc = FB_SLAB / (nv * rs), nms = (no + mc - 1) / mc;
        const int c0 = sp * no * nms / ns, c1 = (sp + 1) * no * nms / ns;
        for (int it = c0; it < c1; ++it) {
            const int n = it / nms, m0 = (it % nms) * mc;
            const int nm = min(mc, no - m0);
            stage(n, m0, nm, 0, nv);
            __syncthreads();
            int b0, b1;
            slice(vpart, vparts, nm * nv, b0, b1);
            for (int mf = b0; mf < b1; ++mf) {
                const int m = mf / nv, f = mf % nv;
                const cd g = Gs[(m * nv + ve) * rs + f];
                cfma(avv, Ts[(m * nv + va) * rs + f], g);
                cfma(avv2, Ts[(m * nv + va2) * rs + f], g);
            }
            __syncthreads();
        }
    }
    __syncthreads();  // every read of the last slab is done
    red[tid] = aoo;
    __syncthreads();
    if (tid < oo) {
        cd sum = make_double2(0.0, 0.0);
        for (int pp = 0; pp < parts; ++pp) sum = cadd(sum, red[pp * oo + tid]);
        Poo[(sp * n3 + blk) * oo + (int64_t)um * no + ui] = cscale(sum, 0.5);
    }
    __syncthreads();
    cd *pv = Pvv + (sp * n3 + ((int64_t)r * N + p) * N + q) * vv;
    red[tid] = avv;
    __syncthreads();
    if (tid < hv) {
        cd sum = make_double2(0.0, 0.0);
        for (int pp = 0; pp < vparts; ++pp) sum = cadd(sum, red[pp * hv + tid]);
        pv[va * nv + ve] = cscale(sum, -0.5);
    }
    __syncthreads();
    red[tid] = avv2;
    __syncthreads();
    if (tid < hv && two) {
        cd sum = make_double2(0.0, 0.0);
        for (int pp = 0; pp < vparts; ++pp) sum = cadd(sum, red[pp * hv + tid]);
        pv[(va + ha) * nv + ve] = cscale(sum, -0.5);
    }
}

// Register-blocked form of k_f_blocks for n_occ <= OM, n_vir <= VM: 256 threads per
// block, the n-slab of the next iteration loaded into registers while the current one is
// used from LDS.  Fvv: a thread owns a 2 x 2 (a, e) tile and a quarter of the m range;
// Foo: a thread owns a 2 x 2 (m, i) tile and one sixteenth of the (e, f) range; each LDS
// read feeds two multiply-adds.  Partial sums are combined through LDS at the end.
template <int OM, int VM, bool EX = false, class IT = cd>
__global__ __launch_bounds__(256) void k_f_blocks_t(SysDev s, const cd *t1, const cd *t2, cd *Poo, cd *Pvv) {
    const IT *oovv = oovv_of<IT>(s);
    static_assert(OM % 8 == 0 && VM % 16 == 0, "tiling");
    // taut(x, n, e, f) and <x n||e f> at x * RX + e * VP + f: rows padded to VP = VM + 1 and
    // row blocks to RX = VM * VP + 1, so that the lanes of one 8-lane group read distinct
    // banks in both role layouts below
    constexpr int VP = VM + 1, RX = VM * VP + 1, SL = OM * RX;
    constexpr int PER = OM * VM * VM / 256;  // slab elements staged per thread
    __shared__ cd TS[SL], GS[SL];
    __shared__ cd T1P[OM * VM], T1Q[OM * VM];  // t1[p], t1[q] for tau's single-amplitude part
    const int N = s.d.N, no = EX ? OM : s.d.no, nv = EX ? VM : s.d.nv;
    const int tid = threadIdx.x;
    const int64_t blk = blockIdx.x;
    const int r = (int)(blk % N), q = (int)((blk / N) % N), p = (int)(blk / ((int64_t)N * N));
    const int kb = kcv(s.kc, N, p, q, r);
    const int64_t base = blk * s.d.t2blk();
    for (int x = tid; x < no * nv; x += 256) {
        T1P[x] = t1[(int64_t)p * no * nv + x];
        T1Q[x] = t1[(int64_t)q * no * nv + x];
    }
    // A slab is loaded as stored (t2 and the integral, with no arithmetic in between, so
    // that every load of the thread is in flight at once) and turned into tau (t1 from LDS)
    // when written to LDS.
    cd pt[PER];
    IT pg[PER];
#define FB_LOAD(n)                                                                              \
    _Pragma("unroll") for (int u = 0; u < PER; ++u) {                                           \
        const int x = tid + 256 * u;                                                            \
        const int row = x / (VM * VM), e = (x / VM) % VM, f = x % VM;                           \
        const bool in_ = row < no && e < nv && f < nv;                                          \
        const int64_t gi = base + (((int64_t)(in_ ? row : 0) * no + (n)) * nv + (in_ ? e : 0)) * nv + (in_ ? f : 0); \
        pt[u] = t2[gi];                                                                         \
        pg[u] = oovv[gi];                                                                       \
    }
#define FB_STORE(n)                                                                             \
    _Pragma("unroll") for (int u = 0; u < PER; ++u) {                                           \
        const int x = tid + 256 * u;                                                            \
        const int row = x / (VM * VM), e = (x / VM) % VM, f = x % VM;                           \
        const bool in_ = row < no && e < nv && f < nv;                                          \
        cd v = pt[u];                                                                           \
        if (in_ && r == p) {                                                                    \
            const cd pp = cmul(T1P[row * nv + e], T1Q[(n) * nv + f]);                           \
            v.x += 0.5 * pp.x;                                                                  \
            v.y += 0.5 * pp.y;                                                                  \
        }                                                                                       \
        if (in_ && kb == p) {                                                                   \
            const cd pp = cmul(T1P[row * nv + f], T1Q[(n) * nv + e]);                           \
            v.x -= 0.5 * pp.x;                                                                  \
            v.y -= 0.5 * pp.y;                                                                  \
        }                                                                                       \
        TS[row * RX + e * VP + f] = in_ ? v : make_double2(0.0, 0.0);                          \
        GS[row * RX + e * VP + f] = in_ ? to_cd(pg[u]) : make_double2(0.0, 0.0);               \
    }
    // Fvv roles: outputs (a0 + 8 da, e0 + 8 de), m quarter; the eight lanes of a group share
    // a0 (one broadcast row) and take eight consecutive e0
    const int vs = tid / 64, vt = tid % 64;
    const int a0 = vt / (VM / 2), e0 = vt % (VM / 2);
    // (VM = 16: 64 tiles of 2 x 2 cover 16 x 16)
    // Foo roles: tile (m0, i0), (e, f) sixteenth
    const int os = tid / 16, ot = tid % 16;
    const int m0 = 2 * (ot / 4), i0 = 2 * (ot % 4);  // OM = 8: 16 tiles of 2 x 2
    cd v00 = {0, 0}, v01 = {0, 0}, v10 = {0, 0}, v11 = {0, 0};
    cd o00 = {0, 0}, o01 = {0, 0}, o10 = {0, 0}, o11 = {0, 0};
    FB_LOAD(0)
    __syncthreads();  // t1 blocks in LDS
    FB_STORE(0)
    __syncthreads();
    for (int n = 0; n < no; ++n) {
        if (n + 1 < no) FB_LOAD(n + 1)
        // Fvv(a,e) += sum_{m in quarter, f} taut(m,n,a,f) <mn||ef>
#pragma unroll
        for (int mm = 0; mm < OM / 4; ++mm) {
            const int m = vs * (OM / 4) + mm;
#pragma unroll 4
            for (int f = 0; f < VM; ++f) {
                const cd ta0 = TS[m * RX + a0 * VP + f], ta1 = TS[m * RX + (a0 + VM / 2) * VP + f];
                const cd ge0 = GS[m * RX + e0 * VP + f], ge1 = GS[m * RX + (e0 + VM / 2) * VP + f];
                cfma(v00, ta0, ge0);
                cfma(v01, ta0, ge1);
                cfma(v10, ta1, ge0);
                cfma(v11, ta1, ge1);
            }
        }
        // Foo(m,i) += sum_{(e,f) in sixteenth} taut(i,n,e,f) <mn||ef>
#pragma unroll 4
        for (int k = 0; k < VM * VM / 16; ++k) {
            const int ef = os * (VM * VM / 16) + k, e = ef / VM, f = ef % VM;
            const cd ti0 = TS[i0 * RX + e * VP + f], ti1 = TS[(i0 + 1) * RX + e * VP + f];
            const cd gm0 = GS[m0 * RX + e * VP + f], gm1 = GS[(m0 + 1) * RX + e * VP + f];
            cfma(o00, ti0, gm0);
            cfma(o01, ti1, gm0);
            cfma(o10, ti0, gm1);
            cfma(o11, ti1, gm1);
        }
        __syncthreads();
        if (n + 1 < no) {
            FB_STORE(n + 1)
        }
        __syncthreads();
    }
#undef FB_LOAD
#undef FB_STORE
    // combine the partial sums (LDS reused)
    cd *ro = TS, *rv = GS;
    ro[os * 64 + ot * 4 + 0] = o00;
    ro[os * 64 + ot * 4 + 1] = o01;
    ro[os * 64 + ot * 4 + 2] = o10;
    ro[os * 64 + ot * 4 + 3] = o11;
    rv[vs * 256 + vt * 4 + 0] = v00;
    rv[vs * 256 + vt * 4 + 1] = v01;
    rv[vs * 256 + vt * 4 + 2] = v10;
    rv[vs * 256 + vt * 4 + 3] = v11;
    __syncthreads();
    if (tid < 64) {
        cd sum = {0, 0};
        for (int k = 0; k < 16; ++k) sum = cadd(sum, ro[k * 64 + tid]);
        const int t = tid / 4, c = tid % 4;
        const int m = 2 * (t / 4) + c / 2, i = 2 * (t % 4) + c % 2;
        if (m < no && i < no) Poo[blk * no * no + (int64_t)m * no + i] = cscale(sum, 0.5);
    }
    {
        cd sum = {0, 0};
        for (int k = 0; k < 4; ++k) sum = cadd(sum, rv[k * 256 + tid]);
        const int t = tid / 4, c = tid % 4;
        const int a = t / (VM / 2) + (VM / 2) * (c / 2), e = t % (VM / 2) + (VM / 2) * (c % 2);
        if (a < nv && e < nv) Pvv[(((int64_t)r * N + p) * N + q) * nv * nv + (int64_t)a * nv + e] = cscale(sum, -0.5);
    }
}

// The two t2-integral sums of the T1 equation read the same t2 block [p,q,r]; one
// workgroup per block stages t2(:, n, :, :), <n q, a p||ef> and <m p, n q||i r, f> through
// LDS one n-slab at a time and forms
//   P1[p][q][r](i,a) += -1/2 sum_{n,e,f} t2(i,n,e,f) <n q, a p || e r, f>   (k = p)
//   P1[r][p][q](i,a) += -1/2 sum_{m,n,f} t2(m,n,a,f) <m p, n q || i r, f>   (k = r)
// written to two partial arrays that k_r1_wave adds.  When the slabs of one n do not fit,
// the two sums take separate passes: the first over slabs of a range of e (every i, a),
// the second over slabs of a range of m (every a, i).  With fr_splits > 1 each pass's list
// of slabs is cut into that many contiguous ranges, one workgroup each (grid splits x N^3),
// and split sp writes slice sp of each partial array.
constexpr int RB_T = 2176, RB_G = 4352, RB_H = 1152;
inline bool r1_blocks_fit(const Dims &d) { return d.no <= 32 && d.nv <= 32; }

constexpr int RB_NT = 1024;
template <class IT>  // element type of the <ov||vv> copy read (complex64 on the mixed path)
__global__ __launch_bounds__(RB_NT) void k_r1_blocks(SysDev s, const cd *t2, cd *P1a, cd *P1b) {
    __shared__ cd Ts[RB_T], Gs[RB_G], Hs[RB_H];
    __shared__ cd red[RB_NT];
    const int N = s.d.N, no = s.d.no, nv = s.d.nv, vv = nv * nv, rs = nv + 1;
    const int tid = threadIdx.x;
    const int64_t n3 = (int64_t)N * N * N;
    const int64_t blk = blockIdx.x % n3;
    const int sp = (int)(blockIdx.x / n3), ns = fr_splits(s.d);
    const int r = (int)(blk % N), q = (int)((blk / N) % N), p = (int)(blk / ((int64_t)N * N));
    const int64_t tb = blk * s.d.t2blk();
    const int64_t ov3 = (int64_t)no * nv * vv, o3v = (int64_t)no * no * no * nv;
    const int64_t gb = blk3(N, q, p, r) * ov3;  // ovvv block [q,p,r]: (n, a, e, f)
    const int64_t hb = blk * o3v;               // ooov block [p,q,r]: (m, n, i, f)
    const int nout = no * nv;                   // outputs (i, a)
    // a thread per output pair (i, a), (i + ho, a): the pair shares its <n q, a p||e r, f>
    // reads in the first sum and its t2 reads in the second
    const int ho = (no + 1) / 2, hout = ho * nv;
    const int parts = RB_NT / hout;             // threads per output pair
    const int part = tid / hout, oi = tid % hout;
    const int ii = oi / nv, aa = oi % nv;
    const bool two = ii + ho < no;              // the second output exists (odd n_occ)
    const int ii2 = two ? ii + ho : ii;         // (a duplicate read otherwise, discarded)
    auto slice = [&](int cnt, int &b0, int &b1) {
        b0 = part < parts ? (int)((int64_t)part * cnt / parts) : 0;
        b1 = part < parts ? (int)((int64_t)(part + 1) * cnt / parts) : 0;
    };
    // t2(x, n, e, f) for rows x0 .. x0+nx-1 and e0 .. e0+ne-1 at ((x - x0) * ne + e - e0) * rs + f
    auto stage_t = [&](int n, int x0, int nx, int e0, int ne) {
        const int per = ne * nv;
#pragma unroll 4
        for (int x = tid; x < nx * per; x += RB_NT) {
            const int row = x / per, e = (x % per) / nv, f = x % nv;
            Ts[(row * ne + e) * rs + f] = t2[tb + (((int64_t)(x0 + row) * no + n) * nv + e0 + e) * nv + f];
        }
    };
    // <m p, n q || i r, f> for m0 .. m0+nm-1 at ((m - m0) * no + i) * rs + f
    auto stage_h = [&](int n, int m0, int nm) {
        for (int x = tid; x < nm * no * nv; x += RB_NT) {
            const int m = x / (no * nv), i = (x / nv) % no, f = x % nv;
            Hs[(m * no + i) * rs + f] = to_cd(ooov_of<IT>(s)[hb + (((int64_t)(m0 + m) * no + n) * no + i) * nv + f]);
        }
    };
    const bool one = (int64_t)no * nv * rs <= RB_T && (int64_t)nv * (vv + 1) <= RB_G && (int64_t)no * no * rs <= RB_H;
    const int ec = one ? nv : min(RB_T / (no * rs), (RB_G / nv - 1) / nv), nes = (nv + ec - 1) / ec;
    cd accA = make_double2(0.0, 0.0), accB = make_double2(0.0, 0.0);
    cd accA2 = make_double2(0.0, 0.0), accB2 = make_double2(0.0, 0.0);
    // this split's range of the slabs (n, e0), n-major
    const int a0 = sp * no * nes / ns, a1 = (sp + 1) * no * nes / ns;
    for (int it = a0; it < a1; ++it) {
        const int n = it / nes, e0 = (it % nes) * ec;
        const int ne = min(ec, nv - e0), per = ne * nv, gs = per + 1;
        stage_t(n, 0, no, e0, ne);
        // <n q, a p || e r, f> for e0 .. e0+ne-1: (a, (e - e0) * nv + f), rows padded to gs
#pragma unroll 4
        for (int x = tid; x < nv * per; x += RB_NT)
            Gs[(x / per) * gs + x % per] =
                to_cd(ovvv_of<IT>(s)[gb + (int64_t)n * nv * vv + (int64_t)(x / per) * vv + e0 * nv + x % per]);
        if (one) stage_h(n, 0, no);
        __syncthreads();
        int b0, b1;
        slice(per, b0, b1);
        for (int ef = b0; ef < b1; ++ef) {
            const cd g = Gs[aa * gs + ef];
            cfma(accA, Ts[(ii * ne + ef / nv) * rs + ef % nv], g);
            cfma(accA2, Ts[(ii2 * ne + ef / nv) * rs + ef % nv], g);
        }
        if (one) {
            slice(no * nv, b0, b1);
            for (int mf = b0; mf < b1; ++mf) {
                const int m = mf / nv, f = mf % nv;
                const cd t = Ts[(m * nv + aa) * rs + f];
                cfma(accB, t, Hs[(m * no + ii) * rs + f]);
                cfma(accB2, t, Hs[(m * no + ii2) * rs + f]);
            }
        }
        __syncthreads();
    }
    if (!one) {
        const int mc = min(min(no, RB_T / (nv * rs)), RB_H / (no * rs)), nms = (no + mc - 1) / mc;
        const int c0 = sp * no * nms / ns, c1 = (sp + 1) * no * nms / ns;
        for (int it = c0; it < c1; ++it) {
            const int n = it / nms, m0 = (it % nms) * mc;
            const int nm = min(mc, no - m0);
            stage_t(n, m0, nm, 0, nv);
            stage_h(n, m0, nm);
            __syncthreads();
            int b0, b1;
            slice(nm * nv, b0, b1);
            for (int mf = b0; mf < b1; ++mf) {
                const int m = mf / nv, f = mf % nv;
                const cd t = Ts[(m * nv + aa) * rs + f];
                cfma(accB, t, Hs[(m * no + ii) * rs + f]);
                cfma(accB2, t, Hs[(m * no + ii2) * rs + f]);
            }
            __syncthreads();
        }
    }
    cd *pa = P1a + (sp * n3 + blk) * nout, *pb = P1b + (sp * n3 + ((int64_t)r * N + p) * N + q) * nout;
    const cd accs[4] = {accA, accA2, accB, accB2};
#pragma unroll
    for (int w = 0; w < 4; ++w) {  // (first sum, i), (first, i + ho), (second, i), (second, i + ho)
        if (w > 0) __syncthreads();
        red[tid] = accs[w];
        __syncthreads();
        if (tid < hout && (w % 2 == 0 || two)) {
            cd sum = make_double2(0.0, 0.0);
            for (int pp = 0; pp < parts; ++pp) sum = cadd(sum, red[pp * hout + tid]);
            (w < 2 ? pa : pb)[(ii + (w % 2) * ho) * nv + aa] = cscale(sum, -0.5);
        }
    }
}

// Register-blocked form of k_r1_blocks for n_occ <= OM, n_vir <= VM: 256 threads per
// block, looping over n with the t2 slab t2(x, n, e, f) and the <m p, n q||i r, f> slab
// staged in LDS (the next n prefetched into registers).  For P1a a thread owns one a and
// a sixteenth of (e, f) and streams <n q, a p||e r, f> from global memory once, for every
// i; for P1b a thread owns one (i, a) and half of the m range.
template <int OM, int VM, bool EX = false, class IT = cd>
__global__ __launch_bounds__(256) void k_r1_blocks_t(SysDev s, const cd *t2, cd *P1a, cd *P1b) {
    static_assert(OM == 8 && VM == 16, "thread roles assume n_occ <= 8, n_vir <= 16");
    constexpr int VP = VM + 1;
    constexpr int TSL = OM * VM * VP, HSL = OM * OM * VP;
    constexpr int PT = OM * VM * VM / 256, PH = OM * OM * VM / 256;
    __shared__ cd TS[TSL];  // t2(x, n, e, f) at (x * VM + e) * VP + f
    __shared__ cd HS[HSL];  // <m p, n q||i r, f> at (m * OM + i) * VP + f
    const int N = s.d.N, no = EX ? OM : s.d.no, nv = EX ? VM : s.d.nv;
    const int tid = threadIdx.x;
    const int64_t blk = blockIdx.x;
    const int r = (int)(blk % N), q = (int)((blk / N) % N), p = (int)(blk / ((int64_t)N * N));
    const int64_t tb = blk * s.d.t2blk();
    const int64_t ov3 = (int64_t)no * nv * nv * nv, o3v = (int64_t)no * no * no * nv;
    const IT *gb = ovvv_of<IT>(s) + blk3(N, q, p, r) * ov3;  // (n, a, e, f)
    const IT *hb = ooov_of<IT>(s) + blk * o3v;               // (m, n, i, f)
    cd pt[PT];
    IT ph[PH];  // in the stored type until written to LDS
#define RB_LOAD(n)                                                                          \
    _Pragma("unroll") for (int u = 0; u < PT; ++u) {                                        \
        const int x = tid + 256 * u, row = x / (VM * VM), e = (x / VM) % VM, f = x % VM;    \
        pt[u] = (row < no && e < nv && f < nv) ? t2[tb + (((int64_t)row * no + (n)) * nv + e) * nv + f] \
                                               : make_double2(0.0, 0.0);                    \
    }                                                                                       \
    _Pragma("unroll") for (int u = 0; u < PH; ++u) {                                        \
        const int x = tid + 256 * u, m = x / (OM * VM), i = (x / VM) % OM, f = x % VM;      \
        ph[u] = (m < no && i < no && f < nv) ? hb[(((int64_t)m * no + (n)) * no + i) * nv + f] \
                                             : IT{};                                        \
    }
#define RB_STORE()                                                                          \
    _Pragma("unroll") for (int u = 0; u < PT; ++u) {                                        \
        const int x = tid + 256 * u, row = x / (VM * VM), e = (x / VM) % VM, f = x % VM;    \
        TS[(row * VM + e) * VP + f] = pt[u];                                                \
    }                                                                                       \
    _Pragma("unroll") for (int u = 0; u < PH; ++u) {                                        \
        const int x = tid + 256 * u, m = x / (OM * VM), i = (x / VM) % OM, f = x % VM;      \
        HS[(m * OM + i) * VP + f] = to_cd(ph[u]);                                           \
    }
    // P1a roles
    const int aa = tid / 16, ks = tid % 16;
    // P1b roles
    const int bi = (tid % 128) / VM, ba = tid % VM, bh = tid / 128;
    cd acc[OM];
#pragma unroll
    for (int i = 0; i < OM; ++i) acc[i] = make_double2(0.0, 0.0);
    cd accb = make_double2(0.0, 0.0);
    RB_LOAD(0)
    RB_STORE()
    __syncthreads();
    using ST = decltype(IT{}.x);
    constexpr int GU = VM * VM / 16;  // integrals of one n per thread
    for (int n = 0; n < no; ++n) {
        // this thread's <n a||e f> of this n first (issued before the next slab's loads, so
        // that waiting for them does not wait for those), all together and without branches,
        // kept as stored until used
        ST gx[GU], gy[GU];
        {
            const IT *g = gb + ((int64_t)n * nv + (aa < nv ? aa : 0)) * nv * nv;
#pragma unroll
            for (int u = 0; u < GU; ++u) {
                const int ef = ks + 16 * u, e = ef / VM, f = ef % VM;
                const IT v = g[e < nv && f < nv ? e * nv + f : 0];
                gx[u] = v.x;
                gy[u] = v.y;
            }
        }
        if (n + 1 < no) RB_LOAD(n + 1)
        // P1a(i, a) += sum_{ef} t2(i,n,e,f) <n a||e f>, this thread's (e, f) = ks + 16 u
        if (aa < nv) {
#pragma unroll
            for (int u = 0; u < GU; ++u) {
                const int ef = ks + 16 * u, e = ef / VM, f = ef % VM;
                if (e < nv && f < nv) {
                    const cd gv = make_double2((double)gx[u], (double)gy[u]);
#pragma unroll
                    for (int i = 0; i < OM; ++i) cfma(acc[i], TS[(i * VM + e) * VP + f], gv);
                }
            }
        }
        // P1b(i, a) += sum_{m in half, f} t2(m,n,a,f) <mn||if>
#pragma unroll
        for (int mm = 0; mm < OM / 2; ++mm) {
            const int m = bh * (OM / 2) + mm;
#pragma unroll 4
            for (int f = 0; f < VM; ++f) cfma(accb, TS[(m * VM + ba) * VP + f], HS[(m * OM + bi) * VP + f]);
        }
        __syncthreads();
        if (n + 1 < no) {
            RB_STORE()
        }
        __syncthreads();
    }
#undef RB_LOAD
#undef RB_STORE
    cd *ra = TS, *rb = HS;  // partial sums (LDS reused)
#pragma unroll
    for (int i = 0; i < OM; ++i) ra[(aa * 16 + ks) * OM + i] = acc[i];
    rb[bh * 128 + (tid % 128)] = accb;
    __syncthreads();
    if (tid < 128) {
        const int i = tid / VM, a = tid % VM;
        cd sa = make_double2(0.0, 0.0);
        for (int k = 0; k < 16; ++k) sa = cadd(sa, ra[(a * 16 + k) * OM + i]);
        const cd sb = cadd(rb[tid], rb[128 + tid]);
        if (i < no && a < nv) {
            P1a[blk * no * nv + (int64_t)i * nv + a] = cscale(sa, -0.5);
            P1b[(((int64_t)r * N + p) * N + q) * no * nv + (int64_t)i * nv + a] = cscale(sb, -0.5);
        }
    }
}

// Foo[k](m,i) = f_mi + 1/2 f_mc t_i^c + sum_{kn} t_n^e <m k,n kn||i k,e kn> + sum_kn Poo
// Fvv[k](a,e) = f_ae - 1/2 f_me t_m^a + sum_{km} t_m^f <a k,m km||e k,f km> + sum_km Pvv
// and the combinations used by the T2 equation:
// Fvt[k](b,f) = Fvv(b,f) - 1/2 t_r^b Fov(r,f),  Fot[k](n,j) = Foo(n,j) + 1/2 t_j^c Fov(n,c)
// One 64-lane wave per output element: the N_k-long sums over the extra momentum and the
// N_k^2 per-block partial sums are spread over the lanes and combined by a wave reduction.
__device__ inline cd wave_sum(cd v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        v.x += __shfl_xor(v.x, o, 64);
        v.y += __shfl_xor(v.y, o, 64);
    }
    return v;
}

// F_ov[k](m,e) = f_me + sum_{kn,n,f} t_{n kn}^{f kn} <m k, n kn || e k, f kn>: one wave per
// output element, the lanes over (kn, n, f) (runs of n_vir contiguous integrals), then a
// fixed-order wave reduction.
template <class IT>
__global__ __launch_bounds__(64) void k_fov(SysDev s, const cd *t1, cd *Fov) {
    const int N = s.d.N, no = s.d.no, nv = s.d.nv, n = no + nv, ov = no * nv;
    const int64_t idx = blockIdx.x;
    const int lane = threadIdx.x;
    const int e = (int)(idx % nv), m = (int)((idx / nv) % no), k = (int)(idx / ((int64_t)no * nv));
    cd acc = make_double2(0.0, 0.0);
    for (int u = lane; u < N * ov; u += 64) {
        const int kn = u / ov, nn = (u / nv) % no, f = u % nv;
        const IT *g = oovv_of<IT>(s) + blk3(N, k, kn, k) * s.d.t2blk() + (int64_t)m * no * nv * nv;
        cfma(acc, t1[(int64_t)u], to_cd(g[((int64_t)nn * nv + e) * nv + f]));
    }
    acc = wave_sum(acc);
    if (lane == 0) Fov[idx] = cadd(s.fock[((int64_t)k * n + m) * n + no + e], acc);
}

template <class IT>
__global__ __launch_bounds__(64) void k_foo_fvv(SysDev s, const cd *t1, const cd *Fov, const cd *Poo,
                                                const cd *Pvv, cd *Foo, cd *Fvv) {
    const int N = s.d.N, no = s.d.no, nv = s.d.nv, n = no + nv;
    const int64_t noo = (int64_t)N * no * no, n3 = (int64_t)N * N * N;
    const int ns = fr_splits(s.d);  // slices of the partial sums
    const int64_t idx = blockIdx.x;
    const int lane = threadIdx.x;
    const int ov = no * nv;
    cd acc = make_double2(0.0, 0.0);
    if (idx < noo) {
        const int i = (int)(idx % no), m = (int)((idx / no) % no), k = (int)(idx / ((int64_t)no * no));
        // sum_{kn, n, e} t_{n kn}^{e kn} <m k, n kn || i k, e kn>
        for (int u = lane; u < N * ov; u += 64) {
            const int kn = u / ov, nn = (u / nv) % no, e = u % nv;
            const IT *g = ooov_of<IT>(s) + blk3(N, k, kn, k) * ((int64_t)no * no * no * nv);
            cfma(acc, t1[((int64_t)kn * no + nn) * nv + e], to_cd(g[(((int64_t)m * no + nn) * no + i) * nv + e]));
        }
        for (int u = lane; u < ns * N * N; u += 64)  // split sp = u / N^2, then the momenta of the block
            acc = cadd(acc, Poo[(((int64_t)(u / (N * N)) * n3 + (int64_t)k * N * N + u % (N * N)) * no + m) * no + i]);
        acc = wave_sum(acc);
        if (lane == 0) {
            const cd *fk = s.fock + (int64_t)k * n * n;
            cd h = make_double2(0.0, 0.0);
            for (int c = 0; c < nv; ++c) cfma(h, fk[m * n + no + c], t1[((int64_t)k * no + i) * nv + c]);
            Foo[idx] = cadd(cadd(fk[m * n + i], cscale(h, 0.5)), acc);
        }
    } else {
        const int64_t r = idx - noo;
        const int e = (int)(r % nv), a = (int)((r / nv) % nv), k = (int)(r / ((int64_t)nv * nv));
        // sum_{km, m, f} t_{m km}^{f km} <a k, m km || e k, f km>, the integral read as
        // -<m km, a k || e k, f km> (ovvv block [km,k,k])
        for (int u = lane; u < N * ov; u += 64) {
            const int km = u / ov, m = (u / nv) % no, f = u % nv;
            const IT *g = ovvv_of<IT>(s) + blk3(N, km, k, k) * ((int64_t)no * nv * nv * nv);
            cfma(acc, t1[((int64_t)km * no + m) * nv + f], to_cd(g[(((int64_t)m * nv + a) * nv + e) * nv + f]));
        }
        acc = make_double2(-acc.x, -acc.y);
        for (int u = lane; u < ns * N * N; u += 64)
            acc = cadd(acc, Pvv[(((int64_t)(u / (N * N)) * n3 + (int64_t)k * N * N + u % (N * N)) * nv + a) * nv + e]);
        acc = wave_sum(acc);
        if (lane == 0) {
            const cd *fk = s.fock + (int64_t)k * n * n;
            cd h = make_double2(0.0, 0.0);
            for (int m = 0; m < no; ++m) cfma(h, fk[m * n + no + e], t1[((int64_t)k * no + m) * nv + a]);
            Fvv[r] = cadd(csub(fk[(no + a) * n + no + e], cscale(h, 0.5)), acc);
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
// canon: only the blocks with ki <= kj and km <= kn (the packed product reads no other)
template <class IT>
__global__ void k_wmnij_init(SysDev s, const cd *t1, cd *WT, bool canon) {
    const int N = s.d.N, no = s.d.no, nv = s.d.nv;
    const int64_t o4 = (int64_t)no * no * no * no, o3v = (int64_t)no * no * no * nv;
    GRID_STRIDE(idx, (int64_t)N * N * N * o4) {
        int nn = (int)(idx % no), m = (int)((idx / no) % no);
        int j = (int)((idx / ((int64_t)no * no)) % no), i = (int)((idx / ((int64_t)no * no * no)) % no);
        int64_t blk = idx / o4;
        int km = (int)(blk % N), kj = (int)((blk / N) % N), ki = (int)(blk / ((int64_t)N * N));
        int kn = kcv(s.kc, N, ki, kj, km);
        if (canon && (ki > kj || km > kn)) continue;
        cd acc = to_cd(oooo_of<IT>(s)[blk3(N, km, kn, ki) * o4 + (((int64_t)m * no + nn) * no + i) * no + j]);
        const IT *g1 = ooov_of<IT>(s) + blk3(N, km, kn, ki) * o3v + (((int64_t)m * no + nn) * no + i) * nv;
        const IT *g2 = ooov_of<IT>(s) + blk3(N, km, kn, kj) * o3v + (((int64_t)m * no + nn) * no + j) * nv;
#pragma unroll 8
        for (int e = 0; e < nv; ++e) {
            cfma(acc, t1[((int64_t)kj * no + j) * nv + e], to_cd(g1[e]));
            cd p = cmul(t1[((int64_t)ki * no + i) * nv + e], to_cd(g2[e]));
            acc = csub(acc, p);
        }
        WT[idx] = acc;
    }
}

// ------------------------------------------------------------------ rearranged hole-hole grouping
// The hole-hole part of the T2 equation in the grouping of Sec. 3.3.4 (eqs. A_3rd, def_X and
// the t2 Y-tilde_{mnij} term of eq. A_4th, with Y-tilde of eq. def_Y_oo), FP64 path.  On
// the W_mnij seed (<mn||ij> + P(ij) t_j^c <mn||ic>, same layout), in place:
//   Y[ki][kj][km](i,j,m,n) = 1/2 seed + 1/2 sum_cd t_i^c t_j^d <mn||cd>   (k_c = k_i, k_d = k_j)
__global__ void k_ytilde(SysDev s, const cd *t1, cd *WT) {
    const int N = s.d.N, no = s.d.no, nv = s.d.nv;
    const int64_t o4 = (int64_t)no * no * no * no;
    GRID_STRIDE(idx, (int64_t)N * N * N * o4) {
        const int nn = (int)(idx % no), m = (int)((idx / no) % no);
        const int j = (int)((idx / ((int64_t)no * no)) % no), i = (int)((idx / ((int64_t)no * no * no)) % no);
        const int64_t blk = idx / o4;
        const int km = (int)(blk % N), kj = (int)((blk / N) % N), ki = (int)(blk / ((int64_t)N * N));
        const int kn = kcv(s.kc, N, ki, kj, km);
        const cd *g = s.oovv + blk3(N, km, kn, ki) * s.d.t2blk() + ((int64_t)m * no + nn) * nv * nv;
        const cd *ti = t1 + ((int64_t)ki * no + i) * nv, *tj = t1 + ((int64_t)kj * no + j) * nv;
        cd acc = make_double2(0.0, 0.0);
        for (int c = 0; c < nv; ++c) {
            cd inner = make_double2(0.0, 0.0);
            for (int dd = 0; dd < nv; ++dd) cfma(inner, tj[dd], g[(int64_t)c * nv + dd]);
            cfma(acc, ti[c], inner);
        }
        const cd w = WT[idx];
        WT[idx] = make_double2(0.5 * (w.x + acc.x), 0.5 * (w.y + acc.y));
    }
}

// The part of the hole-hole ladder 1/2 tau_mn^ab W_mnij carried by tau's single-amplitude
// products, which the t2-only products of the rearranged grouping leave out: with
// W = 2 Y + 1/2 X-tilde (X-tilde = t2 <mn||ef>) and the antisymmetry of W in (m, n),
//   r2[ki][kj][ka](i,j,a,b) += sum_mn t_{m ka}^a t_{n kb}^b W[ki][kj][ka](i,j,m,n)
__global__ void k_hh_t1_rest(SysDev s, const cd *t1, const cd *Y, const cd *X, cd *r2) {
    const int N = s.d.N, no = s.d.no, nv = s.d.nv;
    const int64_t o4 = (int64_t)no * no * no * no;
    GRID_STRIDE(idx, s.d.t2()) {
        const int b = (int)(idx % nv), a = (int)((idx / nv) % nv);
        const int j = (int)((idx / ((int64_t)nv * nv)) % no), i = (int)((idx / ((int64_t)nv * nv * no)) % no);
        const int64_t blk = idx / s.d.t2blk();
        const int ka = (int)(blk % N), kj = (int)((blk / N) % N), ki = (int)(blk / ((int64_t)N * N));
        const int kb = kcv(s.kc, N, ki, kj, ka);
        const int64_t wb = blk * o4 + ((int64_t)i * no + j) * no * no;
        cd acc = make_double2(0.0, 0.0);
        for (int m = 0; m < no; ++m) {
            cd inner = make_double2(0.0, 0.0);
            for (int nn = 0; nn < no; ++nn) {
                const cd y = Y[wb + m * no + nn], x = X[wb + m * no + nn];
                const cd w = make_double2(2.0 * y.x + 0.5 * x.x, 2.0 * y.y + 0.5 * x.y);
                cfma(inner, t1[((int64_t)kb * no + nn) * nv + b], w);
            }
            cfma(acc, t1[((int64_t)ka * no + m) * nv + a], inner);
        }
        r2[idx] = cadd(r2[idx], acc);
    }
}

// Blocked form for n_occ <= OM, n_vir <= VM: one workgroup per (ki, kj, km, m) stages
// <mn||ie> for all (n, i, e) (ki block) and for all (n, j, e) (kj block), <mn||ij> and
// both t1 blocks in LDS, so every ooov / oooo element is read once with contiguous loads;
// a thread owns (n, i) and two j.  LDS rows are padded to n_vir + 1 and ordered so that
// the lanes of a wave (consecutive n, then i) read distinct banks.
template <int OM, int VM, bool EX = false, class IT = cd>
__global__ __launch_bounds__(256) void k_wmnij_init_t(SysDev s, const cd *t1, cd *WT, bool canon);

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
// For fixed (ka, kb, ke, e) this is a rank-o update of the v x v x v slab (a, b, f):
// one workgroup per (ka, kb, ke, e), XCD-contiguous order.  G1(m,a,f) = <m kb, a ka||e f>
// (shared by every b) and t_{m ka}^a go through LDS; a thread owns (b, f), keeps
// <m ka, b kb||e f> and t_{m kb}^b for all m in registers and runs over a.  G1 holds as
// many a at a time as fit DR_G1 elements (all of them when o v^2 <= DR_G1); <ab||ef> is
// read once, <mb||ef> once per such chunk of a, all reads are runs of v.
constexpr int DR_G1 = 2048, DR_T1 = 512;
__host__ __device__ inline bool dress_fits(const Dims &d) {
    return d.no <= 32 && (int64_t)d.no * d.nv <= DR_G1;
}
// register arrays of OM (>= n_occ) entries; OM = 0 selects the plain global-memory path
inline int dress_om(const Dims &d) {
    if (!dress_fits(d)) return 0;
    return d.no <= 8 ? 8 : d.no <= 16 ? 16 : d.no <= 32 ? 32 : 0;
}

template <int OM>
__global__ __launch_bounds__(256) void k_vvvv_dress_t(SysDev s, const cd *t1, cd *Vt) {
    __shared__ cd G1[DR_G1];
    __shared__ cd TA[DR_T1];
    const int N = s.d.N, no = s.d.no, nv = s.d.nv, vv = nv * nv;
    const int64_t v3 = (int64_t)vv * nv, v4 = v3 * nv, ov3 = (int64_t)no * v3;
    const int64_t nblk = (int64_t)N * N * N * nv;
    const int64_t L = xcd_block(nblk);
    if (L >= nblk) return;
    const int e = (int)(L % nv);
    const int64_t blk = L / nv;
    const int ke = (int)(blk % N), kb = (int)((blk / N) % N), ka = (int)(blk / ((int64_t)N * N));
    // <m kb, a ka || e f> at (m, a, f) and <m ka, b kb || e f> at (m, b, f)
    const cd *g1b = s.ovvv + blk3(N, kb, ka, ke) * ov3 + (int64_t)e * nv;
    const cd *g2b = s.ovvv + blk3(N, ka, kb, ke) * ov3 + (int64_t)e * nv;
    const cd *ta = t1 + (int64_t)ka * no * nv, *tb = t1 + (int64_t)kb * no * nv;
    const cd *vb = s.vvvv + blk * v4 + (int64_t)e * nv;
    const int64_t ob = blk * v4 + (int64_t)e * nv;
    if constexpr (OM > 0) {
        // <m kb, a ka||e f> staged for ac values of a at a time: no * ac * nv <= DR_G1 and
        // no * ac <= DR_T1
        const int ac = min(min(nv, DR_G1 / (no * nv)), DR_T1 / no);
        for (int a0 = 0; a0 < nv; a0 += ac) {
            const int na = min(ac, nv - a0), anv = na * nv;
            if (a0) __syncthreads();
            for (int x = threadIdx.x; x < no * anv; x += blockDim.x) {
                const int m = x / anv, af = x % anv;
                G1[x] = g1b[(int64_t)m * v3 + (int64_t)(a0 + af / nv) * vv + af % nv];
            }
            for (int x = threadIdx.x; x < no * na; x += blockDim.x) TA[x] = ta[(x / na) * nv + a0 + x % na];
            __syncthreads();
            for (int bf = threadIdx.x; bf < vv; bf += blockDim.x) {
                const int b = bf / nv, f = bf % nv;
                cd g2[OM], t1b[OM];
#pragma unroll
                for (int m = 0; m < OM; ++m) {
                    g2[m] = m < no ? g2b[(int64_t)m * v3 + (int64_t)b * vv + f] : make_double2(0.0, 0.0);
                    t1b[m] = m < no ? tb[m * nv + b] : make_double2(0.0, 0.0);
                }
                for (int a = 0; a < na; ++a) {
                    const int64_t idx = ob + (int64_t)(a0 + a) * v3 + (int64_t)b * vv + f;
                    cd acc = vb[(int64_t)(a0 + a) * v3 + (int64_t)b * vv + f];
#pragma unroll
                    for (int m = 0; m < OM; ++m) {
                        if (m < no) {
                            cfma(acc, t1b[m], G1[(m * na + a) * nv + f]);
                            acc = csub(acc, cmul(TA[m * na + a], g2[m]));
                        }
                    }
                    Vt[idx] = acc;
                }
            }
        }
    } else {
        for (int bf = threadIdx.x; bf < vv; bf += blockDim.x) {
            const int b = bf / nv, f = bf % nv;
            for (int a = 0; a < nv; ++a) {
                const int64_t idx = ob + (int64_t)a * v3 + (int64_t)b * vv + f;
                cd acc = vb[(int64_t)a * v3 + (int64_t)b * vv + f];
                for (int m = 0; m < no; ++m) {
                    cfma(acc, tb[m * nv + b], g1b[(int64_t)m * v3 + (int64_t)a * vv + f]);
                    acc = csub(acc, cmul(ta[m * nv + a], g2b[(int64_t)m * v3 + (int64_t)b * vv + f]));
                }
                Vt[idx] = acc;
            }
        }
    }
}

// ------------------------------------------------------------------ ring intermediate seed
// ovvoT[km][kb][ke](m,b,j,e) = <m km, b kb || e ke, j kj>: the static ovvo class with its
// last two indices swapped, made once per set of inputs so that every ring seed below
// reads contiguous runs.
template <class OT>
__global__ void k_ovvo_transpose(Dims d, const cd *ovvo, OT *ovvoT) {
    const int no = d.no, nv = d.nv;
    GRID_STRIDE(idx, d.t2()) {
        int e = (int)(idx % nv), j = (int)((idx / nv) % no);
        int64_t mb = idx / ((int64_t)no * nv);  // (block, m, b)
        from_cd(ovvo[(mb * nv + e) * no + j], ovvoT[idx]);
    }
}

// Last-two-index swaps of the static ovvv and oovv classes, so that the contractions over
// their last index below read along lanes:  ovvvT[..](m,b,f,e) = <mb||ef>,
// oovvT[..](m,n,f,e) = <mn||ef>.
// (OT = cf: rounded to complex64, the copy the mixed-precision path reads)
template <class OT>
__global__ void k_swap_last2(int64_t nblocks, int v, const cd *src, OT *dst) {
    const int64_t vv = (int64_t)v * v;
    GRID_STRIDE(idx, nblocks * vv) {
        const int64_t r = idx / vv;
        const int e = (int)(idx % v), f = (int)((idx / v) % v);
        from_cd(src[r * vv + (int64_t)e * v + f], dst[idx]);
    }
}
__global__ void k_to_c64(int64_t n, const cd *src, cf *dst) {
    GRID_STRIDE(idx, n) from_cd(src[idx], dst[idx]);
}
__global__ void k_to_c128(int64_t n, const cf *src, cd *dst) {
    GRID_STRIDE(idx, n) dst[idx] = to_cd(src[idx]);
}

// Z[km][kb][ke](m,n,j,e) = <m km, n kb || e ke, j kj> + sum_f t_j^f <m km, n kb || e ke, f kj>
template <class IT>
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
        cd acc = to_cd(ooov_of<IT>(s)[blk3(N, km, kb, kj) * o3v + (((int64_t)m * no + nn) * no + j) * nv + e]);
        acc = make_double2(-acc.x, -acc.y);
        const IT *g = oovvT_of<IT>(s) + blk * s.d.t2blk() + ((int64_t)m * no + nn) * nv * nv + e;
        #pragma unroll 8
        for (int f = 0; f < nv; ++f) cfma(acc, t1[((int64_t)kj * no + j) * nv + f], to_cd(g[(int64_t)f * nv]));
        Z[idx] = acc;
    }
}

// WR[q][kj][km](j,b,m,e) = <mb||ej> + t_j^f <mb||ef> - t_n^b Z(m,n,j,e)   (t2 part by GEMM)
template <class IT>
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
        cd acc = to_cd(ovvoT_of<IT>(s)[bb * s.d.t2blk() + (((int64_t)m * nv + b) * no + j) * nv + e]);
        const IT *g = ovvvT_of<IT>(s) + bb * ov3 + ((int64_t)m * nv + b) * nv * nv + e;
        #pragma unroll 8
        for (int f = 0; f < nv; ++f) cfma(acc, t1[((int64_t)kj * no + j) * nv + f], to_cd(g[(int64_t)f * nv]));
        const cd *z = Z + bb * o3v + (int64_t)m * no * no * nv + (int64_t)j * nv + e;
        #pragma unroll 8
        for (int nn = 0; nn < no; ++nn)
            acc = csub(acc, cmul(t1[((int64_t)kb * no + nn) * nv + b], z[(int64_t)nn * no * nv]));
        WR[idx] = acc;
    }
}

// Q[ka][kb][ki](m,i,j,b) = sum_e t_i^e <m ka, b kb || e ki, j kj> + 1/2 conj(<i ki, j kj || m ka, b kb>)
template <class IT>
__global__ void k_ring_q(SysDev s, const cd *t1, cd *Q) {
    const int N = s.d.N, no = s.d.no, nv = s.d.nv;
    const int64_t o3v = (int64_t)no * no * no * nv;
    GRID_STRIDE(idx, (int64_t)N * N * N * o3v) {
        int b = (int)(idx % nv), j = (int)((idx / nv) % no);
        int i = (int)((idx / ((int64_t)nv * no)) % no), m = (int)((idx / ((int64_t)nv * no * no)) % no);
        int64_t blk = idx / o3v;
        int ki = (int)(blk % N), kb = (int)((blk / N) % N), ka = (int)(blk / ((int64_t)N * N));
        int kj = kcv(s.kc, N, ka, kb, ki);
        const IT *g = ovvoT_of<IT>(s) + blk * s.d.t2blk() + (((int64_t)m * nv + b) * no + j) * nv;
        cd acc = make_double2(0.0, 0.0);
        #pragma unroll 8
        for (int e = 0; e < nv; ++e) cfma(acc, t1[((int64_t)ki * no + i) * nv + e], to_cd(g[e]));
        cd h = to_cd(ooov_of<IT>(s)[blk3(N, ki, kj, ka) * o3v + (((int64_t)i * no + j) * no + m) * nv + b]);
        acc.x += 0.5 * h.x;
        acc.y -= 0.5 * h.y;
        Q[idx] = acc;
    }
}

// Blocked forms of the three seeds above for n_occ <= OM, n_vir <= VM: one workgroup per
// (momentum block, m), XCD-contiguous order.  Each thread keeps the integral row it
// contracts (over f or e) in registers (for n_vir > 16 the W0 seed keeps one accumulator
// per j instead) and produces the outputs of every j (or i), so every <oo||vv>, <ov||vv>
// and <ov||vo> element is read once instead of n_occ times.
template <int OM, int VM, bool EX = false, class IT = cd>
__global__ __launch_bounds__(OM * VM) void k_ring_z_t(SysDev s, const cd *__restrict__ t1, cd *__restrict__ Z) {
    const int N = s.d.N, no = EX ? OM : s.d.no, nv = EX ? VM : s.d.nv;
    const int64_t o3v = (int64_t)no * no * no * nv;
    const int64_t nblk = (int64_t)N * N * N * no;
    const int64_t L = xcd_block(nblk);
    if (L >= nblk) return;
    const int m = (int)(L % no);
    const int64_t blk = L / no;
    const int ke = (int)(blk % N), kb = (int)((blk / N) % N), km = (int)(blk / ((int64_t)N * N));
    const int kj = kcv(s.kc, N, km, kb, ke);
    const cd *T1J = t1 + (int64_t)kj * no * nv;  // read at wave-uniform addresses (scalar loads)
    const int ne = threadIdx.x;
    if (ne >= no * nv) return;
    const int nn = ne / nv, e = ne % nv;
    const IT *g = oovvT_of<IT>(s) + blk * s.d.t2blk() + ((int64_t)m * no + nn) * nv * nv + e;
    cd gr[VM];
#pragma unroll
    for (int f = 0; f < VM; ++f) gr[f] = f < nv ? to_cd(g[(int64_t)f * nv]) : make_double2(0.0, 0.0);
    const IT *h = ooov_of<IT>(s) + blk3(N, km, kb, kj) * o3v + ((int64_t)m * no + nn) * no * nv + e;
    cd *z = Z + blk * o3v + ((int64_t)m * no + nn) * no * nv + e;
    // the <mn||je> of every j loaded together before any is used (component arrays, clamped
    // addresses), so the thread waits for one memory round trip instead of one per j
    using ST = decltype(IT{}.x);
    ST hx[OM], hy[OM];
#pragma unroll
    for (int j = 0; j < OM; ++j) {
        const IT v = h[(int64_t)(j < no ? j : 0) * nv];
        hx[j] = v.x;
        hy[j] = v.y;
    }
#pragma unroll
    for (int j = 0; j < OM; ++j) {
        if (j >= no) break;
        // <mn||ej> = -<mn||je>
        cd acc = make_double2(-(double)hx[j], -(double)hy[j]);
#pragma unroll
        for (int f = 0; f < VM; ++f)
            if (f < nv) cfma(acc, T1J[j * nv + f], gr[f]);
        z[(int64_t)j * nv] = acc;
    }
}

template <int OM, int VM, bool EX = false, class IT = cd>
__global__ __launch_bounds__(VM * VM) void k_ring_w0_t(SysDev s, const cd *__restrict__ t1, const cd *__restrict__ Z,
                                                      cd *__restrict__ WR) {
    __shared__ cd ZS[OM * OM * VM];  // Z(m, n, j, e) of this m at (n * no + j) * nv + e
    __shared__ cd T1S[VM <= 16 && OM <= 8 ? OM * VM : 1];  // t1[kj](j, f) (n_occ <= 8, n_vir <= 16)
    const int N = s.d.N, no = EX ? OM : s.d.no, nv = EX ? VM : s.d.nv;
    const int64_t ov = (int64_t)no * nv, blkq = ov * ov;
    const int64_t o3v = (int64_t)no * no * no * nv, ov3 = (int64_t)no * nv * nv * nv;
    const int64_t nblk = (int64_t)N * N * N * no;
    const int64_t L = xcd_block(nblk);
    if (L >= nblk) return;
    const int m = (int)(L % no);
    const int64_t blk = L / no;  // (q, kj, km)
    const int km = (int)(blk % N), kj = (int)((blk / N) % N), q = (int)(blk / ((int64_t)N * N));
    const int kb = kcv(s.kc, N, kj, 0, q), ke = kcv(s.kc, N, km, 0, q);
    const int64_t bb = blk3(N, km, kb, ke);
    const cd *zb = Z + bb * o3v + (int64_t)m * no * no * nv;
    const cd *T1J = t1 + (int64_t)kj * no * nv;  // t1[kj](j, f)
    const int be = threadIdx.x;
    const bool act = be < nv * nv;
    const int b = act ? be / nv : 0, e = act ? be % nv : 0;
    const IT *g = ovvvT_of<IT>(s) + bb * ov3 + ((int64_t)m * nv + b) * nv * nv + e;
    const IT *w0 = ovvoT_of<IT>(s) + bb * s.d.t2blk() + ((int64_t)m * nv + b) * no * nv + e;
    cd *wr = WR + blk * blkq + (int64_t)b * ov + (int64_t)m * nv + e;
    if constexpr (VM <= 16 && OM <= 8) {
        // Every global operand of the thread (the row <m b||f e> over f, <m b||e j> over j,
        // t1 at kb) is loaded before the shared slabs and before any use, so all of them are
        // in flight together (converted element by element, they would each take a full
        // memory round trip); then one j at a time, the stored values converted on use.
        // (component arrays: an array of the HIP vector structs would be kept in memory)
        constexpr int NT = VM * VM, ZN = (OM * OM * VM + NT - 1) / NT;
        const int nz = no * no * nv;
        double zx[ZN], zy[ZN];
#pragma unroll
        for (int u = 0; u < ZN; ++u) {  // the Z slab first: its LDS stores wait for it alone
            const int x = threadIdx.x + u * NT;
            const cd v = zb[x < nz ? x : 0];
            zx[u] = v.x;
            zy[u] = v.y;
        }
        const cd t1v = T1J[threadIdx.x < no * nv ? threadIdx.x : 0];
        using ST = decltype(IT{}.x);
        ST gx[VM], gy[VM], wx[OM], wy[OM];
        double tx[OM], ty[OM];
#pragma unroll
        for (int f = 0; f < VM; ++f) {
            const IT v = g[(int64_t)(act && f < nv ? f : 0) * nv];
            gx[f] = act && f < nv ? v.x : ST(0);
            gy[f] = act && f < nv ? v.y : ST(0);
        }
#pragma unroll
        for (int j = 0; j < OM; ++j) {
            const IT v = w0[(int64_t)(act && j < no ? j : 0) * nv];
            wx[j] = v.x;
            wy[j] = v.y;
        }
#pragma unroll
        for (int n = 0; n < OM; ++n) {
            const cd v = t1[((int64_t)kb * no + (n < no ? n : 0)) * nv + b];
            tx[n] = v.x;
            ty[n] = v.y;
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int u = 0; u < ZN; ++u) {
            const int x = threadIdx.x + u * NT;
            if (x < nz) ZS[x] = make_double2(zx[u], zy[u]);
        }
        if (threadIdx.x < no * nv) T1S[threadIdx.x] = t1v;
        __syncthreads();
        if (!act) return;
#pragma unroll
        for (int j = 0; j < OM; ++j) {
            if (j >= no) break;
            cd acc = make_double2((double)wx[j], (double)wy[j]);
#pragma unroll
            for (int f = 0; f < VM; ++f)
                if (f < nv) cfma(acc, T1S[j * nv + f], make_double2((double)gx[f], (double)gy[f]));
#pragma unroll
            for (int n = 0; n < OM; ++n)
                if (n < no) acc = csub(acc, cmul(make_double2(tx[n], ty[n]), ZS[(n * no + j) * nv + e]));
            wr[(int64_t)j * nv * ov] = acc;
        }
        return;
    }
    for (int x = threadIdx.x; x < no * no * nv; x += blockDim.x) ZS[x] = zb[x];
    __syncthreads();
    if (!act) return;
    if constexpr (VM <= 16) {
        // the row <m b||f e> over f in registers, one j at a time
        cd gr[VM], tb[OM];
#pragma unroll
        for (int f = 0; f < VM; ++f) gr[f] = f < nv ? to_cd(g[(int64_t)f * nv]) : make_double2(0.0, 0.0);
#pragma unroll
        for (int n = 0; n < OM; ++n) tb[n] = n < no ? t1[((int64_t)kb * no + n) * nv + b] : make_double2(0.0, 0.0);
        for (int j = 0; j < no; ++j) {
            cd acc = to_cd(w0[(int64_t)j * nv]);
#pragma unroll
            for (int f = 0; f < VM; ++f)
                if (f < nv) cfma(acc, T1J[j * nv + f], gr[f]);
#pragma unroll
            for (int n = 0; n < OM; ++n)
                if (n < no) acc = csub(acc, cmul(tb[n], ZS[(n * no + j) * nv + e]));
            wr[(int64_t)j * nv * ov] = acc;
        }
        return;
    }
    // wider rows: one accumulator per j, each <m b||f e> loaded once and used for every j
    cd acc[OM];
#pragma unroll
    for (int j = 0; j < OM; ++j) acc[j] = j < no ? to_cd(w0[(int64_t)j * nv]) : make_double2(0.0, 0.0);
#pragma unroll
    for (int f = 0; f < VM; ++f) {
        if (f >= nv) break;
        const cd gv = to_cd(g[(int64_t)f * nv]);
#pragma unroll
        for (int j = 0; j < OM; ++j)
            if (j < no) cfma(acc[j], T1J[j * nv + f], gv);
    }
#pragma unroll
    for (int n = 0; n < OM; ++n) {
        if (n >= no) break;
        const cd tv = t1[((int64_t)kb * no + n) * nv + b];
#pragma unroll
        for (int j = 0; j < OM; ++j)
            if (j < no) acc[j] = csub(acc[j], cmul(tv, ZS[(n * no + j) * nv + e]));
    }
#pragma unroll
    for (int j = 0; j < OM; ++j)
        if (j < no) wr[(int64_t)j * nv * ov] = acc[j];
}

template <int OM, int VM, bool EX = false, class IT = cd, int IC = OM>
__global__ __launch_bounds__(OM * VM) void k_ring_q_t(SysDev s, const cd *t1, cd *Q) {
    // The <m b||e j> slab of this m goes through LDS EP values of e at a time (so that
    // many workgroups fit on a CU), at e * (no * nv + 1) + j * nv + b: a lane (j, b) reads
    // consecutive words, and the staging writes (consecutive e) are one padded row apart.
    // The next phase's slab is loaded into registers while the current one is used.  A
    // workgroup forms the outputs of IC values of i (i0 .. i0 + IC - 1): with IC < OM the
    // i range is shared by several workgroups, each reading the slab, so that a thread
    // keeps IC accumulators in registers.
    constexpr int EP = 4;
    constexpr int NT = OM * VM;
    __shared__ cd GS[EP * (OM * VM + 1)];
    __shared__ cd T1I[OM * VM];  // t1[ki](i, e)
    const int N = s.d.N, no = EX ? OM : s.d.no, nv = EX ? VM : s.d.nv, rp = no * nv + 1;
    const int64_t o3v = (int64_t)no * no * no * nv;
    const int nh = (no + IC - 1) / IC;
    const int64_t nblk = (int64_t)N * N * N * no * nh;
    const int64_t L0 = xcd_block(nblk);
    if (L0 >= nblk) return;
    const int i0 = (int)(L0 % nh) * IC;
    const int64_t L = L0 / nh;
    const int m = (int)(L % no);
    const int64_t blk = L / no;
    const int ki = (int)(blk % N), kb = (int)((blk / N) % N), ka = (int)(blk / ((int64_t)N * N));
    const int kj = kcv(s.kc, N, ka, kb, ki);
    const IT *gb = ovvoT_of<IT>(s) + blk * s.d.t2blk() + (int64_t)m * nv * no * nv;  // (b, j, e)
    const int nph = no * nv * EP;  // staged elements per phase
    IT st[EP];  // in the stored type until written to LDS, so the load is not waited for early
    auto load_phase = [&](int e0) {
#pragma unroll
        for (int u = 0; u < EP; ++u) {
            const int x = threadIdx.x + u * NT;  // (bj, el) with el fastest
            const int bj = x / EP, e = e0 + x % EP;
            st[u] = x < nph && e < nv ? gb[(int64_t)bj * nv + e] : IT{};
        }
    };
    auto store_phase = [&]() {
#pragma unroll
        for (int u = 0; u < EP; ++u) {
            const int x = threadIdx.x + u * NT, bj = x / EP, el = x % EP;
            if (x < nph) GS[el * rp + (bj % no) * nv + bj / no] = to_cd(st[u]);
        }
    };
    load_phase(0);
    for (int x = threadIdx.x; x < no * nv; x += blockDim.x) T1I[x] = t1[(int64_t)ki * no * nv + x];
    const int jb = threadIdx.x;
    const bool act = jb < no * nv;
    cd acc[IC];
#pragma unroll
    for (int i = 0; i < IC; ++i) acc[i] = make_double2(0.0, 0.0);
    for (int e0 = 0; e0 < nv; e0 += EP) {
        if (e0 > 0) __syncthreads();  // every read of the previous phase is done
        store_phase();
        __syncthreads();
        if (e0 + EP < nv) load_phase(e0 + EP);
        if (act) {
#pragma unroll
            for (int el = 0; el < EP; ++el) {
                if (e0 + el >= nv) break;
                const cd g = GS[el * rp + jb];
#pragma unroll
                for (int i = 0; i < IC; ++i)
                    if (i0 + i < no) cfma(acc[i], T1I[(i0 + i) * nv + e0 + el], g);
            }
        }
    }
    if (!act) return;
    const int j = jb / nv, b = jb % nv;
    const IT *h = ooov_of<IT>(s) + blk3(N, ki, kj, ka) * o3v + ((int64_t)j * no + m) * nv + b;
    cd *qo = Q + blk * o3v + (int64_t)m * no * no * nv + jb;
#pragma unroll
    for (int ic = 0; ic < IC; ++ic) {
        const int i = i0 + ic;
        if (i >= no) break;
        const cd x = to_cd(h[(int64_t)i * no * no * nv]);
        cd v = acc[ic];
        v.x += 0.5 * x.x;
        v.y -= 0.5 * x.y;
        qo[(int64_t)i * no * nv] = v;
    }
}

// X[q][ki][kj](i,a,j,b), k_a = k_i + q, k_b = k_j - q: everything of the T2 equation that is
// neither the driver nor a ladder, arranged so that one P(ij)P(ab) produces it:
//   - t_i^e t_m^a <mb||ej>                       (ring, the t2 W_mbej part is added by GEMM)
//   - 1/2 t_i^c <ab||cj>,  - 1/2 t_r^a <rb||ij>  (antisymmetric in ab / in ij, so 1/2 under
//                                                 P(ij)P(ab) gives P(ij) / -P(ab) of them)
//   + 1/2 t_ij^af Fvt(b,f), - 1/2 t_in^ab Fot(n,j) (antisymmetric in ij / in ab, likewise)
// This uses the antisymmetry of t2 in (i,j) and (a,b).
template <class IT>
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
        const IT *g = ovvv_of<IT>(s) + blk3(N, kj, ki, ka) * ov3 + (int64_t)j * nv * nv * nv + (int64_t)a * nv + b;
        #pragma unroll 8
        for (int c = 0; c < nv; ++c) cfma(y, t1[((int64_t)ki * no + i) * nv + c], cconj(to_cd(g[(int64_t)c * nv * nv])));
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

// The t1 x Q term of the X seed for the 16-row tiles, written to X before k_xinit_t adds
// the others: X[q,ki,kj](i, a, j, b) = -sum_m t_m^a(ka) Q[ka,kb,ki](m, i, j, b).  A workgroup
// per (X block, i, range of 256 (j, b)); the thread of (j, b) keeps Q(m, i, j, b) for every m
// in registers and forms every a, so each Q element is read once (inside k_xinit_t each of
// the n_vir workgroups of a block would read the whole o^3 v slab again); t1 at
// wave-uniform addresses.
template <int OM>
__global__ __launch_bounds__(256) void k_xinit_q(SysDev s, const cd *__restrict__ t1, const cd *__restrict__ Q,
                                                 cd *__restrict__ X) {
    const int N = s.d.N, no = s.d.no, nv = s.d.nv;
    const int64_t ov = (int64_t)no * nv, o3v = ov * no * no;
    const int nch = (int)((ov + 255) / 256);
    const int64_t nblk = (int64_t)N * N * N * no * nch;
    const int64_t L = xcd_block(nblk);
    if (L >= nblk) return;
    const int ch = (int)(L % nch), i = (int)((L / nch) % no);
    const int64_t blk = L / ((int64_t)nch * no);  // (q, ki, kj) as in k_xinit_t
    const int kj = (int)(blk % N), ki = (int)((blk / N) % N), q = (int)(blk / ((int64_t)N * N));
    const int ka = kcv(s.kc, N, ki, q, 0), kb = kcv(s.kc, N, kj, 0, q);
    const int jb = ch * 256 + threadIdx.x;
    if (jb >= ov) return;
    const cd *qb = Q + blk3(N, ka, kb, ki) * o3v + (int64_t)i * ov + jb;
    cd qm[OM];
#pragma unroll
    for (int m = 0; m < OM; ++m) qm[m] = m < no ? qb[(int64_t)m * no * ov] : make_double2(0.0, 0.0);
    const cd *ta = t1 + (int64_t)ka * no * nv;
    cd *xb = X + blk * ov * ov + (int64_t)i * nv * ov + jb;
    for (int a = 0; a < nv; ++a) {
        cd acc = make_double2(0.0, 0.0);
#pragma unroll
        for (int m = 0; m < OM; ++m)
            if (m < no) cfma(acc, ta[m * nv + a], qm[m]);
        xb[(int64_t)a * ov] = make_double2(-acc.x, -acc.y);
    }
}

// The same X seed in one blocked pass for n_occ <= OM, n_vir <= VM: a workgroup per
// (q, ki, kj, a) in XCD-contiguous order, a thread per (j, b) holding the no values of X at
// (i, a, j, b) for every i.  Every <ov||vv> and t2 element is read once (t2 of this a goes
// through LDS, with each (i, n) run of b contiguous, a half of the i at a time (a quarter
// for 16-row tiles) so that more workgroups fit on a CU; its loads are issued before the integral terms and land in LDS
// after them); the Q slab of (ka, kb, ki) is shared by the nv workgroups of one (q, ki, kj),
// which run next to each other on one XCD, so it comes from L2 after the first.  t1 is read
// at wave-uniform addresses (scalar loads).  The coefficients -1, -1/2, 1/2, -1/2 of the four
// terms are folded into one factor of each product (exact scalings), so one accumulator per
// i takes all of them.  With 16-row tiles the t1 x Q term is already in X (k_xinit_q) and
// the accumulators start from it.
template <int OM, int VM, bool EX = false, class IT = cd>
__global__ __launch_bounds__(OM * VM) void k_xinit_t(SysDev s, const cd *t1, const cd *t2, const cd *Q,
                                                    const cd *Fot, const cd *Fvt, cd *X) {
    constexpr bool QX = OM > 8;                  // the t1 x Q term is in X already
    constexpr int NPH = OM > 8 ? 4 : 2;          // LDS phases over i
    constexpr int IH = (OM + NPH - 1) / NPH;  // i values per phase
    constexpr int NT = OM * VM;       // threads
    __shared__ cd T2S[IH * OM * (VM + 1)];  // t2[ki,kj,ka](i0 + il, n, a, b) at (il * no + n) * (nv + 1) + b
    __shared__ cd FV[VM * VM];        // 1/2 Fvt[kb](b, f) at f * nv + b
    __shared__ cd FO[OM * OM];        // -1/2 Fot[kj](n, j)
    const int N = s.d.N, no = EX ? OM : s.d.no, nv = EX ? VM : s.d.nv;
    const int64_t ov = (int64_t)no * nv, ov3 = ov * nv * nv, o3v = ov * no * no;
    const int64_t nblk = (int64_t)N * N * N * nv;
    const int64_t L = xcd_block(nblk);
    if (L >= nblk) return;
    const int a = (int)(L % nv);
    const int64_t blk = L / nv;  // (q, ki, kj)
    const int kj = (int)(blk % N), ki = (int)((blk / N) % N), q = (int)(blk / ((int64_t)N * N));
    const int ka = kcv(s.kc, N, ki, q, 0), kb = kcv(s.kc, N, kj, 0, q);
    const cd *tb = t2 + blk3(N, ki, kj, ka) * s.d.t2blk() + (int64_t)a * nv;
    const int nh = IH * no * nv;  // staged elements per phase
    cd st[IH];
    auto load_half = [&](int i0) {
#pragma unroll
        for (int u = 0; u < IH; ++u) {
            const int x = threadIdx.x + u * NT, il = x / (no * nv), i = i0 + il;
            st[u] = x < nh && i < no ? tb[((int64_t)i * no + (x / nv) % no) * nv * nv + x % nv] : make_double2(0.0, 0.0);
        }
    };
    const int vp = nv + 1;  // padded rows: the lanes of different j read different banks
    auto store_half = [&]() {
#pragma unroll
        for (int u = 0; u < IH; ++u) {
            const int x = threadIdx.x + u * NT;
            if (x < nh) T2S[(x / nv) * vp + x % nv] = st[u];
        }
    };
    load_half(0);
    for (int x = threadIdx.x; x < nv * nv; x += blockDim.x)
        FV[(x % nv) * nv + x / nv] = cscale(Fvt[(int64_t)kb * nv * nv + x], 0.5);
    for (int x = threadIdx.x; x < no * no; x += blockDim.x) FO[x] = cscale(Fot[(int64_t)kj * no * no + x], -0.5);
    const int jb = threadIdx.x;
    const bool act = jb < no * nv;
    const int j = act ? jb / nv : 0, b = act ? jb % nv : 0;
    cd acc[OM];
#pragma unroll
    for (int i = 0; i < OM; ++i) acc[i] = make_double2(0.0, 0.0);
    if constexpr (QX) {
        if (act) {
            const cd *x0 = X + blk * ov * ov + (int64_t)a * ov + jb;
#pragma unroll
            for (int i = 0; i < OM; ++i)
                if (i < no) acc[i] = x0[(int64_t)i * nv * ov];
        }
    }
    if (act) {
        // -1/2 sum_c t_i^c conj(<j kj, c ki || a ka, b kb>)
        const IT *gb = ovvv_of<IT>(s) + blk3(N, kj, ki, ka) * ov3 + (int64_t)j * nv * nv * nv + (int64_t)a * nv + b;
        const cd *t1i = t1 + (int64_t)ki * no * nv;
#pragma unroll
        for (int c = 0; c < VM; ++c) {
            if (c >= nv) break;
            const cd gv = to_cd(gb[(int64_t)c * nv * nv]);
            const cd g = make_double2(-0.5 * gv.x, 0.5 * gv.y);  // -1/2 conj(<..>)
#pragma unroll
            for (int i = 0; i < OM; ++i)
                if (i < no) cfma(acc[i], t1i[i * nv + c], g);
        }
        // -sum_m t_m^a Q(m, i, j, b)
        const cd *qb = Q + blk3(N, ka, kb, ki) * o3v + jb;
#pragma unroll
        for (int m = 0; m < OM; ++m) {
            if (QX || m >= no) break;
            const cd tv = t1[((int64_t)ka * no + m) * nv + a];
            const cd tm = make_double2(-tv.x, -tv.y);
#pragma unroll
            for (int i = 0; i < OM; ++i)
                if (i < no) cfma(acc[i], tm, qb[(int64_t)(m * no + i) * ov]);
        }
    }
    store_half();
#pragma unroll
    for (int p = 0; p < NPH; ++p) {
        const int i0 = p * IH;
        if (i0 >= no) break;
        if (p > 0) {
            load_half(i0);
            __syncthreads();  // every read of the previous phase is done
            store_half();
        }
        __syncthreads();
        if (act) {
            // +1/2 sum_f t_ij^af Fvt[kb](b, f)
#pragma unroll
            for (int f = 0; f < VM; ++f) {
                if (f >= nv) break;
                const cd fv = FV[f * nv + b];
#pragma unroll
                for (int il = 0; il < IH; ++il)
                    if (i0 + il < no) cfma(acc[i0 + il], T2S[(il * no + j) * vp + f], fv);
            }
            // -1/2 sum_n t_in^ab Fot[kj](n, j)
#pragma unroll
            for (int n = 0; n < OM; ++n) {
                if (n >= no) break;
                const cd fo = FO[n * no + j];
#pragma unroll
                for (int il = 0; il < IH; ++il)
                    if (i0 + il < no) cfma(acc[i0 + il], T2S[(il * no + n) * vp + b], fo);
            }
        }
    }
    if (!act) return;
    cd *xb = X + blk * ov * ov + (int64_t)a * ov + jb;
#pragma unroll
    for (int i = 0; i < OM; ++i)
        if (i < no) xb[(int64_t)i * nv * ov] = acc[i];
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
template <class IT>
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
            const IT *g = ovvv_of<IT>(s) + blk3(N, kx, k, ky) * ov3 + (int64_t)a * nv * nv;
            for (int nn = 0; nn < no; ++nn)
                for (int ef = 0; ef < nv * nv; ++ef)
                    acc = csub(acc, cmul(t[(int64_t)nn * nv * nv + ef], to_cd(g[(int64_t)nn * nv * nv * nv + ef])));
        }
        {
            const cd *t = t2 + blk3(N, kx, ky, k) * s.d.t2blk() + (int64_t)a * nv;
            const IT *g = ooov_of<IT>(s) + blk3(N, kx, ky, k) * o3v + (int64_t)i * nv;
            for (int mm = 0; mm < no; ++mm)
                for (int nn = 0; nn < no; ++nn)
                    for (int f = 0; f < nv; ++f)
                        acc = csub(acc, cmul(t[((int64_t)mm * no + nn) * nv * nv + f],
                                             to_cd(g[((int64_t)mm * no + nn) * no * nv + f])));
        }
        P1[idx] = cscale(acc, 0.5);
    }
}

// r1 = conj(f_ia) + t_i^c Fvv(a,c) - t_r^a Foo(r,i) + sum_kn t2[k,kn,k](i,n,a,f) Fov[kn](n,f)
//      + sum_kn t_r^c <a k, r kn||i k, c kn> + sum_kx P1
// One 64-lane wave per output (k, i, a): the N_k-long sums over kn and
// the N_k^2 partial sums are spread over the lanes (consecutive lanes read consecutive
// elements) and combined by a wave reduction, so the kernel is not limited by a few
// hundred threads each running the whole sum.
template <class IT>
__global__ __launch_bounds__(64) void k_r1_wave(SysDev s, const cd *t1, const cd *t2, const cd *Foo, const cd *Fvv,
                                                const cd *Fov, const cd *P1, int nparts, cd *r1) {
    const int N = s.d.N, no = s.d.no, nv = s.d.nv, n = no + nv;
    const int64_t idx = blockIdx.x;
    const int a = (int)(idx % nv), i = (int)((idx / nv) % no), k = (int)(idx / ((int64_t)no * nv));
    const int lane = threadIdx.x;
    const int ov = no * nv;
    cd acc = make_double2(0.0, 0.0);
    // sum_{kn, n, f} t_{i k, n kn}^{a k, f kn} F(n kn, f kn)
    for (int u = lane; u < N * ov; u += 64) {
        const int kn = u / ov, nn = (u / nv) % no, f = u % nv;
        const cd *t = t2 + blk3(N, k, kn, k) * s.d.t2blk() + (int64_t)i * no * nv * nv + (int64_t)a * nv;
        cfma(acc, t[(int64_t)nn * nv * nv + f], Fov[((int64_t)kn * no + nn) * nv + f]);
    }
    // sum_{kn, r, c} t_{r kn}^{c kn} <r kn, a k || c kn, i k>   (ovvo block [kn,k,kn], read
    // from its copy with the last two indices swapped, ovvoT(r, a, i, c))
    for (int u = lane; u < N * ov; u += 64) {
        const int kn = u / ov, r = (u / nv) % no, c = u % nv;
        const IT *g = ovvoT_of<IT>(s) + blk3(N, kn, k, kn) * s.d.t2blk() + ((int64_t)a * no + i) * nv + c;
        cfma(acc, t1[((int64_t)kn * no + r) * nv + c], to_cd(g[(int64_t)r * nv * no * nv]));
    }
    // the per-block partial sums
    const int64_t np = (int64_t)N * N * N * no * nv;
    for (int u = lane; u < nparts * N * N; u += 64) {
        const int pp = u / (N * N), kk = u % (N * N);
        acc = cadd(acc, P1[pp * np + (((int64_t)k * N * N + kk) * no + i) * nv + a]);
    }
    acc = wave_sum(acc);
    if (lane == 0) {
        cd v = cconj(s.fock[((int64_t)k * n + i) * n + no + a]);
        for (int c = 0; c < nv; ++c) cfma(v, t1[((int64_t)k * no + i) * nv + c], Fvv[((int64_t)k * nv + a) * nv + c]);
        for (int r = 0; r < no; ++r)
            v = csub(v, cmul(t1[((int64_t)k * no + r) * nv + a], Foo[((int64_t)k * no + r) * no + i]));
        r1[idx] = cadd(v, acc);
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

// the blocked side kernels at the workload's exact block shape (n_occ = 8, n_vir = 16) take
// the sizes as constants (every bound check folds away and index divisions become shifts),
// with the element type of the integral copies a kernel reads (complex64 on the
// mixed-precision path)
#define LAUNCH_TI(K, grid, block, ...)                                                    \
    do {                                                                                  \
        if (s.ovvv_c) {                                                                   \
            if (s.d.no == 8 && s.d.nv == 16)                                              \
                hipLaunchKernelGGL((K<8, 16, true, cf>), grid, block, 0, st, __VA_ARGS__);  \
            else                                                                          \
                hipLaunchKernelGGL((K<8, 16, false, cf>), grid, block, 0, st, __VA_ARGS__); \
        } else {                                                                          \
            if (s.d.no == 8 && s.d.nv == 16)                                              \
                hipLaunchKernelGGL((K<8, 16, true, cd>), grid, block, 0, st, __VA_ARGS__);  \
            else                                                                          \
                hipLaunchKernelGGL((K<8, 16, false, cd>), grid, block, 0, st, __VA_ARGS__); \
        }                                                                                 \
        CK_CHECK(hipGetLastError());                                                      \
    } while (0)
// a wider tile (OMV x VMV, sizes as run-time values), with the element type of the copies
#define LAUNCH_WI(OMV, VMV, K, grid, block, ...)                                             \
    do {                                                                                  \
        if (s.ovvv_c)                                                                     \
            hipLaunchKernelGGL((K<OMV, VMV, false, cf>), grid, block, 0, st, __VA_ARGS__);  \
        else                                                                              \
            hipLaunchKernelGGL((K<OMV, VMV, false, cd>), grid, block, 0, st, __VA_ARGS__);  \
        CK_CHECK(hipGetLastError());                                                      \
    } while (0)
#define LAUNCH_32I(K, grid, block, ...) LAUNCH_WI(8, 32, K, grid, block, __VA_ARGS__)

void launch_f(const SysDev &s, const cd *t1, const cd *t2, FWork w, hipStream_t st) {
    const int64_t N = s.d.N, no = s.d.no, nv = s.d.nv;
    if (s.ovvv_c)
        hipLaunchKernelGGL(k_fov<cf>, dim3((unsigned)(N * no * nv)), dim3(64), 0, st, s, t1, w.Fov);
    else
        hipLaunchKernelGGL(k_fov<cd>, dim3((unsigned)(N * no * nv)), dim3(64), 0, st, s, t1, w.Fov);
    CK_CHECK(hipGetLastError());
    if (no <= 8 && nv <= 16) {
        LAUNCH_TI(k_f_blocks_t, dim3((unsigned)(N * N * N)), dim3(256), s, t1, t2, w.Poo, w.Pvv);
    } else if (bsum_rb_fits(s.d)) {
        launch_f_blocks_rb(s, t1, t2, w.Poo, w.Pvv, st);
    } else if (f_blocks_fit(s.d)) {
        const dim3 grid((unsigned)(N * N * N * fr_splits(s.d)));
        if (s.oovv_c)
            hipLaunchKernelGGL(k_f_blocks<cf>, grid, dim3(FB_NT), 0, st, s, t1, t2, w.Poo, w.Pvv);
        else
            hipLaunchKernelGGL(k_f_blocks<cd>, grid, dim3(FB_NT), 0, st, s, t1, t2, w.Poo, w.Pvv);
        CK_CHECK(hipGetLastError());
    } else if (s.ovvv_c) {
        LAUNCH(k_foo_partial<cf>, N * N * N * no * no, s, t1, t2, w.Poo);
        LAUNCH(k_fvv_partial<cf>, N * N * N * nv * nv, s, t1, t2, w.Pvv);
    } else {
        LAUNCH(k_foo_partial<cd>, N * N * N * no * no, s, t1, t2, w.Poo);
        LAUNCH(k_fvv_partial<cd>, N * N * N * nv * nv, s, t1, t2, w.Pvv);
    }
    const dim3 gf((unsigned)(N * no * no + N * nv * nv));
    if (s.ovvv_c)
        hipLaunchKernelGGL(k_foo_fvv<cf>, gf, dim3(64), 0, st, s, t1, w.Fov, w.Poo, w.Pvv, w.Foo, w.Fvv);
    else
        hipLaunchKernelGGL(k_foo_fvv<cd>, gf, dim3(64), 0, st, s, t1, w.Fov, w.Poo, w.Pvv, w.Foo, w.Fvv);
    CK_CHECK(hipGetLastError());
    LAUNCH(k_ftilde, N * no * no + N * nv * nv, s.d, t1, w.Foo, w.Fvv, w.Fov, w.Fot, w.Fvt);
}

template <int OM, int VM, bool EX, class IT>
__global__ __launch_bounds__(256) void k_wmnij_init_t(SysDev s, const cd *t1, cd *WT, bool canon) {
    static_assert(OM == 8, "thread roles assume n_occ <= 8");
    constexpr int VP = VM + 1;
    __shared__ cd A1[OM * OM * VP];  // <m km, n kn||i ki, e> at (i * OM + n) * VP + e
    __shared__ cd A2[OM * OM * VP];  // <m km, n kn||j kj, e> at (j * OM + n) * VP + e
    __shared__ cd T1I[OM * VP], T1J[OM * VP];
    __shared__ cd O4[OM * OM * OM];  // <m km, n kn||i ki, j kj> at (n * OM + i) * OM + j
    const int N = s.d.N, no = EX ? OM : s.d.no, nv = EX ? VM : s.d.nv;
    const int64_t o4 = (int64_t)no * no * no * no, o3v = (int64_t)no * no * no * nv;
    const int64_t nblk = (int64_t)N * N * N * no;
    // canon: only blocks holding canonical (ki, i, j) rows and (km, m, n) columns (ki <= kj,
    // km <= kn) are needed; the others exit, and plain launch order spreads the rest evenly
    // over the XCDs
    const int64_t L = canon ? (int64_t)blockIdx.x : xcd_block(nblk);
    if (L >= nblk) return;
    const int m = (int)(L % no);
    const int64_t blk = L / no;
    const int km = (int)(blk % N), kj = (int)((blk / N) % N), ki = (int)(blk / ((int64_t)N * N));
    const int kn = kcv(s.kc, N, ki, kj, km);
    if (canon && (ki > kj || km > kn)) return;
    const IT *g1 = ooov_of<IT>(s) + blk3(N, km, kn, ki) * o3v + (int64_t)m * no * no * nv;  // (n, i, e)
    const IT *g2 = ooov_of<IT>(s) + blk3(N, km, kn, kj) * o3v + (int64_t)m * no * no * nv;  // (n, j, e)
    const IT *g0 = oooo_of<IT>(s) + blk3(N, km, kn, ki) * o4 + (int64_t)m * no * no * no;    // (n, i, j)
    for (int x = threadIdx.x; x < no * no * nv; x += blockDim.x) {
        const int n = x / (no * nv), i = (x / nv) % no, e = x % nv;
        A1[(i * OM + n) * VP + e] = to_cd(g1[x]);
        A2[(i * OM + n) * VP + e] = to_cd(g2[x]);
    }
    for (int x = threadIdx.x; x < no * nv; x += blockDim.x) {
        T1I[(x / nv) * VP + x % nv] = t1[(int64_t)ki * no * nv + x];
        T1J[(x / nv) * VP + x % nv] = t1[(int64_t)kj * no * nv + x];
    }
    for (int x = threadIdx.x; x < no * no * no; x += blockDim.x) {
        const int n = x / (no * no), i = (x / no) % no, j = x % no;
        O4[(n * OM + i) * OM + j] = to_cd(g0[x]);
    }
    __syncthreads();
    const int n = threadIdx.x % OM, i = (threadIdx.x / OM) % OM, j0 = 2 * (threadIdx.x / (OM * OM));
    if (n >= no || i >= no) return;
    cd *wt = WT + blk * o4 + (int64_t)m * no + n;
#pragma unroll
    for (int jj = 0; jj < 2; ++jj) {
        const int j = j0 + jj;
        if (j >= no) continue;
        cd acc = O4[(n * OM + i) * OM + j];
#pragma unroll
        for (int e = 0; e < VM; ++e)
            if (e < nv) {
                cfma(acc, T1J[j * VP + e], A1[(i * OM + n) * VP + e]);
                acc = csub(acc, cmul(T1I[i * VP + e], A2[(j * OM + n) * VP + e]));
            }
        wt[((int64_t)i * no + j) * no * no] = acc;
    }
}

void launch_wmnij_init(const SysDev &s, const cd *t1, cd *WT, bool canon, hipStream_t st) {
    const int64_t N = s.d.N, no = s.d.no, nv = s.d.nv;
    if (no <= 8 && nv <= 16) {
        LAUNCH_TI(k_wmnij_init_t, xcd_grid(N * N * N * no), dim3(256), s, t1, WT, canon);
    } else if (s.ovvv_c) {
        LAUNCH(k_wmnij_init<cf>, N * N * N * no * no * no * no, s, t1, WT, canon);
    } else {
        LAUNCH(k_wmnij_init<cd>, N * N * N * no * no * no * no, s, t1, WT, canon);
    }
}

void launch_block_transpose(const Dims &d, const cd *src, cd *dst, hipStream_t st) {
    const int R = d.no * d.no, C = d.nv * d.nv;
    dim3 g((unsigned)((int64_t)((R + 31) / 32) * ((C + 31) / 32) * d.N * d.N * d.N));
    hipLaunchKernelGGL(k_block_transpose, g, dim3(256), 0, st, d, src, dst);
    CK_CHECK(hipGetLastError());
}

// Y-tilde in two steps for n_occ <= OM, n_vir <= VM: a workgroup per (ki, kj, km, m) in
// XCD-contiguous order stages the <mn||cd> rows of its m (every n, c, d; the block has
// k_c = k_i and k_d = k_j) and both t1 blocks in LDS, forms
//   Z(n, i, d) = sum_c t_i^c <mn||cd>
// in LDS, then Y(i, j, m, n) = 1/2 seed + 1/2 sum_d Z(n, i, d) t_j^d for every (i, j, n).
// o^3 v^2 + o^4 v complex MACs per block instead of o^4 v^2, and every <oo||vv> element is
// read once: ((ki, kj, km) -> (km, kn, ki) is one to one).
template <int OM, int VM>
__global__ __launch_bounds__(256) void k_ytilde_t(SysDev s, const cd *t1, cd *WT) {
    constexpr int VP = VM + 1;
    __shared__ cd G[OM * VM * VP];   // <m n||c d> at (n * nv + c) * VP + d
    __shared__ cd Z[OM * OM * VP];   // Z(n, i, d) at (n * no + i) * VP + d
    __shared__ cd TI[OM * VM], TJ[OM * VM];
    const int N = s.d.N, no = s.d.no, nv = s.d.nv;
    const int64_t o4 = (int64_t)no * no * no * no;
    const int64_t nwg = (int64_t)N * N * N * no;
    const int64_t L = xcd_block(nwg);
    if (L >= nwg) return;
    const int m = (int)(L % no);
    const int64_t blk = L / no;
    const int km = (int)(blk % N), kj = (int)((blk / N) % N), ki = (int)(blk / ((int64_t)N * N));
    const int kn = kcv(s.kc, N, ki, kj, km);
    const cd *g = s.oovv + blk3(N, km, kn, ki) * s.d.t2blk() + (int64_t)m * no * nv * nv;
    const int ovv = no * nv * nv;
    for (int x = threadIdx.x; x < ovv; x += blockDim.x) G[(x / nv) * VP + x % nv] = g[x];
    for (int x = threadIdx.x; x < no * nv; x += blockDim.x) {
        TI[x] = t1[(int64_t)ki * no * nv + x];
        TJ[x] = t1[(int64_t)kj * no * nv + x];
    }
    __syncthreads();
    for (int x = threadIdx.x; x < no * no * nv; x += blockDim.x) {  // (n, i, d), d fastest
        const int d = x % nv, i = (x / nv) % no, n = x / (nv * no);
        cd acc = make_double2(0.0, 0.0);
        for (int c = 0; c < nv; ++c) cfma(acc, TI[i * nv + c], G[(n * nv + c) * VP + d]);
        Z[(n * no + i) * VP + d] = acc;
    }
    __syncthreads();
    cd *wb = WT + blk * o4 + (int64_t)m * no;
    for (int x = threadIdx.x; x < no * no * no; x += blockDim.x) {  // (i, j, n), n fastest
        const int n = x % no, j = (x / no) % no, i = x / (no * no);
        cd acc = make_double2(0.0, 0.0);
        for (int d = 0; d < nv; ++d) cfma(acc, Z[(n * no + i) * VP + d], TJ[j * nv + d]);
        cd *w = wb + ((int64_t)i * no + j) * no * no + n;
        const cd v = *w;
        *w = make_double2(0.5 * (v.x + acc.x), 0.5 * (v.y + acc.y));
    }
}

// The single-amplitude rest of the hole-hole ladder in two steps for n_occ <= OM,
// n_vir <= VM: a workgroup per (ki, kj, ka, i) stages W(j, m, n) = 2 Y + 1/2 X-tilde of its i
// and both t1 blocks in LDS, forms U(j, m, b) = sum_n W(j, m, n) t_{n kb}^b in LDS, then adds
// sum_m t_{m ka}^a U(j, m, b) to r2(i, j, a, b) for every (j, a, b), a contiguous o v^2 run.
template <int OM, int VM>
__global__ __launch_bounds__(256) void k_hh_t1_rest_t(SysDev s, const cd *t1, const cd *Y, const cd *X, cd *r2) {
    constexpr int OP = OM + 1, VP = VM + 1;
    __shared__ cd W[OM * OM * OP];   // W(j, m, n) at (j * no + m) * OP + n
    __shared__ cd U[OM * OM * VP];   // U(j, m, b) at (j * no + m) * VP + b
    __shared__ cd TA[OM * VM], TB[OM * VM];
    const int N = s.d.N, no = s.d.no, nv = s.d.nv;
    const int64_t o4 = (int64_t)no * no * no * no;
    const int64_t nwg = (int64_t)N * N * N * no;
    const int64_t L = xcd_block(nwg);
    if (L >= nwg) return;
    const int i = (int)(L % no);
    const int64_t blk = L / no;
    const int ka = (int)(blk % N), kj = (int)((blk / N) % N), ki = (int)(blk / ((int64_t)N * N));
    const int kb = kcv(s.kc, N, ki, kj, ka);
    const int o3 = no * no * no;
    const int64_t wb = blk * o4 + (int64_t)i * o3;
    for (int x = threadIdx.x; x < o3; x += blockDim.x) {
        const cd y = Y[wb + x], xt = X[wb + x];
        W[(x / no) * OP + x % no] = make_double2(2.0 * y.x + 0.5 * xt.x, 2.0 * y.y + 0.5 * xt.y);
    }
    for (int x = threadIdx.x; x < no * nv; x += blockDim.x) {
        TA[x] = t1[(int64_t)ka * no * nv + x];
        TB[x] = t1[(int64_t)kb * no * nv + x];
    }
    __syncthreads();
    for (int x = threadIdx.x; x < no * no * nv; x += blockDim.x) {  // (j, m, b), b fastest
        const int b = x % nv, jm = x / nv;
        cd acc = make_double2(0.0, 0.0);
        for (int n = 0; n < no; ++n) cfma(acc, W[jm * OP + n], TB[n * nv + b]);
        U[jm * VP + b] = acc;
    }
    __syncthreads();
    cd *rb = r2 + blk * s.d.t2blk() + (int64_t)i * no * nv * nv;
    for (int x = threadIdx.x; x < no * nv * nv; x += blockDim.x) {  // (j, a, b), b fastest
        const int b = x % nv, a = (x / nv) % nv, j = x / (nv * nv);
        cd acc = make_double2(0.0, 0.0);
        for (int mm = 0; mm < no; ++mm) cfma(acc, TA[mm * nv + a], U[(j * no + mm) * VP + b]);
        rb[x] = cadd(rb[x], acc);
    }
}

void launch_ytilde(const SysDev &s, const cd *t1, cd *WT, hipStream_t st) {
    const int64_t N = s.d.N, no = s.d.no;
    if (no <= 8 && s.d.nv <= 16) {
        hipLaunchKernelGGL((k_ytilde_t<8, 16>), xcd_grid(N * N * N * no), dim3(256), 0, st, s, t1, WT);
        CK_CHECK(hipGetLastError());
        return;
    }
    LAUNCH(k_ytilde, N * N * N * no * no * no * no, s, t1, WT);
}

void launch_hh_t1_rest(const SysDev &s, const cd *t1, const cd *Y, const cd *X, cd *r2, hipStream_t st) {
    const int64_t N = s.d.N, no = s.d.no;
    if (no <= 8 && s.d.nv <= 16) {
        hipLaunchKernelGGL((k_hh_t1_rest_t<8, 16>), xcd_grid(N * N * N * no), dim3(256), 0, st, s, t1, Y, X, r2);
        CK_CHECK(hipGetLastError());
        return;
    }
    LAUNCH(k_hh_t1_rest, s.d.t2(), s, t1, Y, X, r2);
}

void launch_vvvv_dress(const SysDev &s, const cd *t1, cd *Vt, hipStream_t st) {
    const int64_t N = s.d.N, nv = s.d.nv;
    const dim3 grid = xcd_grid(N * N * N * nv);
    switch (dress_om(s.d)) {
    case 8: hipLaunchKernelGGL((k_vvvv_dress_t<8>), grid, dim3(256), 0, st, s, t1, Vt); break;
    case 16: hipLaunchKernelGGL((k_vvvv_dress_t<16>), grid, dim3(256), 0, st, s, t1, Vt); break;
    case 32: hipLaunchKernelGGL((k_vvvv_dress_t<32>), grid, dim3(256), 0, st, s, t1, Vt); break;
    default: hipLaunchKernelGGL((k_vvvv_dress_t<0>), grid, dim3(256), 0, st, s, t1, Vt); break;
    }
    CK_CHECK(hipGetLastError());
}

void launch_static_copies(const SysDev &s, const StaticCopies &c, hipStream_t st) {
    const int64_t N3 = (int64_t)s.d.N * s.d.N * s.d.N, o = s.d.no, v = s.d.nv;
    LAUNCH(k_ovvo_transpose<cd>, s.d.t2(), s.d, s.ovvo, c.ovvoT);
    LAUNCH(k_swap_last2<cd>, N3 * o * v * v * v, N3 * o * v, (int)v, s.ovvv, c.ovvvT);
    LAUNCH(k_swap_last2<cd>, N3 * o * o * v * v, N3 * o * o, (int)v, s.oovv, c.oovvT);
}

void launch_round_c64(int64_t n, const cd *src, cf *dst, hipStream_t st) { LAUNCH(k_to_c64, n, n, src, dst); }
void launch_to_c128(int64_t n, const cf *src, cd *dst, hipStream_t st) { LAUNCH(k_to_c128, n, n, src, dst); }
void launch_swap_last2_c64(int64_t nblocks, int v, const cd *src, cf *dst, hipStream_t st) {
    LAUNCH(k_swap_last2<cf>, nblocks * v * v, nblocks, v, src, dst);
}
void launch_ovvo_transpose_c64(const Dims &d, const cd *ovvo, cf *ovvoT, hipStream_t st) {
    LAUNCH(k_ovvo_transpose<cf>, d.t2(), d, ovvo, ovvoT);
}

// The W_mbej seed: Z into scratch, then W0 (reads Z) into WR.
void launch_ring_w(const SysDev &s, const cd *t1, cd *scratch, cd *WR, hipStream_t st) {
    const int64_t N = s.d.N, no = s.d.no, nv = s.d.nv;
    const int64_t n3 = N * N * N;
    if (no <= 8 && nv <= 16) {
        const dim3 grid = xcd_grid(n3 * no);
        LAUNCH_TI(k_ring_z_t, grid, dim3(8 * 16), s, t1, scratch);
        LAUNCH_TI(k_ring_w0_t, grid, dim3(16 * 16), s, t1, scratch, WR);
    } else if (no <= 8 && nv <= 32) {
        const dim3 grid = xcd_grid(n3 * no);
        LAUNCH_32I(k_ring_z_t, grid, dim3(8 * 32), s, t1, scratch);
        LAUNCH_32I(k_ring_w0_t, grid, dim3(32 * 32), s, t1, scratch, WR);
    } else if (no <= 16 && nv <= 16) {
        const dim3 grid = xcd_grid(n3 * no);
        LAUNCH_WI(16, 16, k_ring_z_t, grid, dim3(16 * 16), s, t1, scratch);
        LAUNCH_WI(16, 16, k_ring_w0_t, grid, dim3(16 * 16), s, t1, scratch, WR);
    } else if (no <= 16 && nv <= 32) {  // the W0 seed's Z slab: 128 KB of LDS, one workgroup per CU
        const dim3 grid = xcd_grid(n3 * no);
        LAUNCH_WI(16, 32, k_ring_z_t, grid, dim3(16 * 32), s, t1, scratch);
        LAUNCH_WI(16, 32, k_ring_w0_t, grid, dim3(32 * 32), s, t1, scratch, WR);
    } else {
        if (s.ovvv_c) {
            LAUNCH(k_ring_z<cf>, n3 * no * no * no * nv, s, t1, scratch);
            LAUNCH(k_ring_w0<cf>, n3 * no * nv * no * nv, s, t1, scratch, WR);
        } else {
            LAUNCH(k_ring_z<cd>, n3 * no * no * no * nv, s, t1, scratch);
            LAUNCH(k_ring_w0<cd>, n3 * no * nv * no * nv, s, t1, scratch, WR);
        }
    }
}

// The X seed: Q into scratch, then the one-pass seed (reads Q, t2 and the F blocks) into X.
void launch_ring_x(const SysDev &s, const cd *t1, const cd *t2, const FWork &w, cd *scratch, cd *X,
                   hipStream_t st) {
    const int64_t N = s.d.N, no = s.d.no, nv = s.d.nv;
    const int64_t n3 = N * N * N;
    if (no <= 8 && nv <= 16) {
        LAUNCH_TI(k_ring_q_t, xcd_grid(n3 * no), dim3(8 * 16), s, t1, scratch);
    } else if (no <= 8 && nv <= 32) {
        LAUNCH_32I(k_ring_q_t, xcd_grid(n3 * no), dim3(8 * 32), s, t1, scratch);
    } else if (no <= 16 && nv <= 32) {
        // 16-row tiles, each workgroup taking half of the i range (eight accumulators per
        // thread; sixteen would spill)
        const dim3 g = xcd_grid(n3 * no * ((no + 7) / 8));
        if (s.ovvv_c)
            hipLaunchKernelGGL((k_ring_q_t<16, 32, false, cf, 8>), g, dim3(16 * 32), 0, st, s, t1, scratch);
        else
            hipLaunchKernelGGL((k_ring_q_t<16, 32, false, cd, 8>), g, dim3(16 * 32), 0, st, s, t1, scratch);
        CK_CHECK(hipGetLastError());
    } else if (s.ovvv_c) {
        LAUNCH(k_ring_q<cf>, n3 * no * no * no * nv, s, t1, scratch);
    } else {
        LAUNCH(k_ring_q<cd>, n3 * no * no * no * nv, s, t1, scratch);
    }
    if (no <= 8 && nv <= 16) {
        LAUNCH_TI(k_xinit_t, xcd_grid(n3 * nv), dim3(8 * 16), s, t1, t2, scratch, w.Fot, w.Fvt, X);
    } else if (no <= 8 && nv <= 32) {
        LAUNCH_32I(k_xinit_t, xcd_grid(n3 * nv), dim3(8 * 32), s, t1, t2, scratch, w.Fot, w.Fvt, X);
    } else if (no <= 16 && nv <= 32) {
        hipLaunchKernelGGL(k_xinit_q<16>, xcd_grid(n3 * no * ((no * nv + 255) / 256)), dim3(256), 0, st, s, t1,
                           scratch, X);
        CK_CHECK(hipGetLastError());
        if (nv <= 16)
            LAUNCH_WI(16, 16, k_xinit_t, xcd_grid(n3 * nv), dim3(16 * 16), s, t1, t2, scratch, w.Fot, w.Fvt, X);
        else
            LAUNCH_WI(16, 32, k_xinit_t, xcd_grid(n3 * nv), dim3(16 * 32), s, t1, t2, scratch, w.Fot, w.Fvt, X);
    } else if (s.ovvv_c) {
        LAUNCH(k_ring_xinit<cf>, n3 * no * nv * no * nv, s, t1, t2, scratch, w.Fot, w.Fvt, X);
    } else {
        LAUNCH(k_ring_xinit<cd>, n3 * no * nv * no * nv, s, t1, t2, scratch, w.Fot, w.Fvt, X);
    }
}

void launch_ring_init(const SysDev &s, const cd *t1, const cd *t2, const FWork &w, cd *scratch, cd *WR, cd *X,
                      hipStream_t st) {
    launch_ring_w(s, t1, scratch, WR, st);
    launch_ring_x(s, t1, t2, w, scratch, X, st);
}

void launch_assemble_r2(const SysDev &s, const cd *X, cd *r2, hipStream_t st) {
    const int64_t N = s.d.N, no = s.d.no;
    hipLaunchKernelGGL(k_assemble_r2, xcd_grid(N * N * N * no * no), dim3(256), 0, st, s, X, r2);
    CK_CHECK(hipGetLastError());
}

// partial arrays of N^3 o v elements that the R1 block sums leave for k_r1_wave
static int r1_parts(const Dims &d) {
    if (d.no <= 8 && d.nv <= 16) return 2;
    return r1_blocks_fit(d) ? 2 * fr_splits(d) : 1;
}

void launch_r1_partials(const SysDev &s, const cd *t2, cd *P1, hipStream_t st) {
    const int64_t N = s.d.N, no = s.d.no, nv = s.d.nv;
    const int64_t np = N * N * N * no * nv;  // P1 holds r1_parts partial arrays of np elements
    if (no <= 8 && nv <= 16) {
        LAUNCH_TI(k_r1_blocks_t, dim3((unsigned)(N * N * N)), dim3(256), s, t2, P1, P1 + np);
    } else if (bsum_rb_fits(s.d)) {
        launch_r1_blocks_rb(s, t2, P1, P1 + fr_splits(s.d) * np, st);
    } else if (r1_blocks_fit(s.d)) {
        const int ns = fr_splits(s.d);
        const dim3 grid((unsigned)(N * N * N * ns));
        if (s.ovvv_c)
            hipLaunchKernelGGL(k_r1_blocks<cf>, grid, dim3(RB_NT), 0, st, s, t2, P1, P1 + ns * np);
        else
            hipLaunchKernelGGL(k_r1_blocks<cd>, grid, dim3(RB_NT), 0, st, s, t2, P1, P1 + ns * np);
        CK_CHECK(hipGetLastError());
    } else if (s.ovvv_c) {
        LAUNCH(k_r1_partial<cf>, N * N * N * no * nv, s, t2, P1);
    } else {
        LAUNCH(k_r1_partial<cd>, N * N * N * no * nv, s, t2, P1);
    }
}

void launch_r1_final(const SysDev &s, const cd *t1, const cd *t2, const FWork &w, const cd *P1, cd *r1,
                     hipStream_t st) {
    const int64_t N = s.d.N, no = s.d.no, nv = s.d.nv;
    if (s.ovvv_c)
        hipLaunchKernelGGL(k_r1_wave<cf>, dim3((unsigned)(N * no * nv)), dim3(64), 0, st, s, t1, t2, w.Foo, w.Fvv,
                           w.Fov, P1, r1_parts(s.d), r1);
    else
        hipLaunchKernelGGL(k_r1_wave<cd>, dim3((unsigned)(N * no * nv)), dim3(64), 0, st, s, t1, t2, w.Foo, w.Fvv,
                           w.Fov, P1, r1_parts(s.d), r1);
    CK_CHECK(hipGetLastError());
}

void launch_r1(const SysDev &s, const cd *t1, const cd *t2, const FWork &w, cd *P1, cd *r1, hipStream_t st) {
    launch_r1_partials(s, t2, P1, st);
    launch_r1_final(s, t1, t2, w, P1, r1, st);
}

}  // namespace ck
