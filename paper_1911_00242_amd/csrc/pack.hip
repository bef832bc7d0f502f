// Antisymmetric pair packing of the ladder operands (mixed-precision path).
//
// tau_{ij}^{ef}, <mn||ef>, the T1-dressed <ab||ef> and W_mnij are antisymmetric under the
// exchange of the two members of a pair (with their momenta), and so is the
// particle-particle / hole-hole ladder contribution to R_{ij}^{ab} in (i, j) and in (a, b).
// Within a group of total pair momentum K, a pair (kx, x; ky, y), ky = K - kx, is canonical
// when (kx, x) < (ky, y) in (momentum, orbital) order.  A sum over all pairs of a product
// of two antisymmetric factors is twice the sum over canonical pairs (the diagonal terms
// vanish), and a result antisymmetric in both pairs is fixed by its canonical rows and
// columns.  The ladder products therefore run on packed operands, canonical pairs of every
// group in a fixed order padded with zeros to a multiple of 16, and take an eighth of the
// work of the full products; their result stays packed (Lp) until the R2 assembly expands
// it.  Every packed operand is written here in the storage of the ladder family: split
// storage, or complex64 when the family's products run on complex64 operands.
#include <algorithm>

#include "common.h"
#include "mixed.h"
#include "pack.h"

namespace ck {

// tau_pk[K][p'][p] = tau_{i ki, j kj}^{e ke, f kf} for canonical (ki, i, j) = p' and canonical
// (ke, e, f) = p of group K (rows ld elements apart; the padding rows are written as zeros).
// A thread per element, consecutive threads on consecutive p, so the reads of t2 and of the
// pair list are contiguous across a wave; the workgroup's 256 elements (32 whole chunks:
// PV is a multiple of 8) are put together in split storage in LDS and written as 16-byte
// words.  EX: n_occ = 8, n_vir = 16 as constants.
template <bool EX>
__global__ __launch_bounds__(256) void k_tau_pack(Dims d, const int32_t *kc, PairTabs pt, const cd *t1,
                                                  const cd *t2, uint16_t *out, int64_t ld, bool c64) {
    __shared__ __align__(16) uint16_t S[256 * 4];  // chunk-local split layout: chunk * 32 + plane * 8 + q
    const int N = d.N, no = EX ? 8 : d.no, nv = EX ? 16 : d.nv;
    const int64_t t2blk = (int64_t)no * no * nv * nv;
    const int64_t total = (int64_t)N * pt.PO * pt.PV;
    for (int64_t x0 = (int64_t)blockIdx.x * 256; x0 < total; x0 += (int64_t)gridDim.x * 256) {
        const int64_t x = x0 + threadIdx.x;
        cd v = make_double2(0.0, 0.0);
        if (x < total) {
            const int64_t row = x / pt.PV;  // K * PO + p'
            const int col = (int)(x - row * pt.PV);
            const int K = (int)(row / pt.PO);
            const int pij = pt.olist[row];
            const int pr = pt.vlist[(int64_t)K * pt.PV + col];
            if (pij >= 0 && pr >= 0) {
                const int ki = pij / (no * no), i = (pij / no) % no, j = pij % no;
                const int kj = kcv(kc, N, K, 0, ki);
                const int ke = pr / (nv * nv), e = (pr / nv) % nv, f = pr % nv;
                const int kf = kcv(kc, N, ki, kj, ke);
                const int64_t idx = blk3(N, ki, kj, ke) * t2blk + (((int64_t)i * no + j) * nv + e) * nv + f;
                v = tau_el(t1, t2, idx, ki, kj, ke, kf, i, j, e, f, no, nv, 1.0);
            }
        }
        if (c64) {  // complex64 storage: consecutive threads write consecutive elements of a row
            if (x < total) {
                const int64_t row = x / pt.PV;
                reinterpret_cast<cf *>(out)[row * ld + (x - row * pt.PV)] = make_float2((float)v.x, (float)v.y);
            }
            continue;  // uniform over the grid: no barrier is skipped by part of a workgroup
        }
        uint16_t h0, h1, h2, h3;
        split2c(v, h0, h1, h2, h3);
        const int ch = threadIdx.x >> 3, q = threadIdx.x & 7;
        S[ch * 32 + q] = h0;
        S[ch * 32 + 8 + q] = h1;
        S[ch * 32 + 16 + q] = h2;
        S[ch * 32 + 24 + q] = h3;
        __syncthreads();
        if (threadIdx.x < 128) {
            const int c = threadIdx.x >> 2, p = threadIdx.x & 3;  // chunk, plane
            const int64_t xc = x0 + c * 8;                        // first element of the chunk
            if (xc < total) {
                const int64_t row = xc / pt.PV;
                const int64_t o = row * ld + (xc - row * pt.PV);
                *(uint4 *)(out + split_index(o, p)) = *(const uint4 *)(S + c * 32 + p * 8);
            }
        }
        __syncthreads();
    }
}

// tauT_pk[K][p'][p] = tau_{m km, n kn}^{a ka, b kb} for canonical (ka, a, b) = p' and
// canonical (km, m, n) = p: the B operand of the hole-hole ladder, which is the tau_pk of
// the same group transposed (padding included).  A workgroup moves a 64 x 64 tile of split
// storage through LDS, each element as one 8-byte unit of its four bf16 planes; both the
// reads and the writes are whole 64-byte chunks.
constexpr int TT = 64;
__global__ __launch_bounds__(256) void k_tau_transpose(int PO, int PV, const uint16_t *src, int64_t lds,
                                                       uint16_t *dst, int64_t ldd) {
    __shared__ uint2 T[TT][TT + 1];  // [p' - m0][p - n0]
    const int K = blockIdx.z, m0 = blockIdx.y * TT, n0 = blockIdx.x * TT;
    for (int u = threadIdx.x; u < TT * (TT / 8); u += blockDim.x) {
        const int r = u / (TT / 8), c = u % (TT / 8), row = m0 + r, col = n0 + c * 8;
        if (row >= PO || col >= PV) continue;
        const uint4 *s = (const uint4 *)(src + split_index(((int64_t)K * PO + row) * lds + col, 0));
        uint32_t w[4][4];
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const uint4 v = s[p];
            w[p][0] = v.x, w[p][1] = v.y, w[p][2] = v.z, w[p][3] = v.w;
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int sh = (q & 1) * 16, k = q >> 1;
            const uint32_t h0 = (w[0][k] >> sh) & 0xffffu, h1 = (w[1][k] >> sh) & 0xffffu;
            const uint32_t h2 = (w[2][k] >> sh) & 0xffffu, h3 = (w[3][k] >> sh) & 0xffffu;
            T[r][c * 8 + q] = make_uint2(h0 | h1 << 16, h2 | h3 << 16);
        }
    }
    __syncthreads();
    for (int u = threadIdx.x; u < TT * (TT / 8); u += blockDim.x) {
        const int r = u / (TT / 8), c = u % (TT / 8), row = n0 + r, col = m0 + c * 8;
        if (row >= PV || col >= PO) continue;
        uint2 e[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) e[q] = T[c * 8 + q][r];
        uint4 *o = (uint4 *)(dst + split_index(((int64_t)K * PV + row) * ldd + col, 0));
        o[0] = make_uint4((e[0].x & 0xffffu) | e[1].x << 16, (e[2].x & 0xffffu) | e[3].x << 16,
                          (e[4].x & 0xffffu) | e[5].x << 16, (e[6].x & 0xffffu) | e[7].x << 16);
        o[1] = make_uint4(e[0].x >> 16 | (e[1].x & 0xffff0000u), e[2].x >> 16 | (e[3].x & 0xffff0000u),
                          e[4].x >> 16 | (e[5].x & 0xffff0000u), e[6].x >> 16 | (e[7].x & 0xffff0000u));
        o[2] = make_uint4((e[0].y & 0xffffu) | e[1].y << 16, (e[2].y & 0xffffu) | e[3].y << 16,
                          (e[4].y & 0xffffu) | e[5].y << 16, (e[6].y & 0xffffu) | e[7].y << 16);
        o[3] = make_uint4(e[0].y >> 16 | (e[1].y & 0xffff0000u), e[2].y >> 16 | (e[3].y & 0xffff0000u),
                          e[4].y >> 16 | (e[5].y & 0xffff0000u), e[6].y >> 16 | (e[7].y & 0xffff0000u));
    }
}

// The same transpose in complex64 storage: 8-byte elements through a 64 x 64 LDS tile.
__global__ __launch_bounds__(256) void k_tau_transpose_c64(int PO, int PV, const uint2 *src, int64_t lds, uint2 *dst,
                                                           int64_t ldd) {
    __shared__ uint2 T[TT][TT + 1];  // [p' - m0][p - n0]
    const int K = blockIdx.z, m0 = blockIdx.y * TT, n0 = blockIdx.x * TT;
    for (int u = threadIdx.x; u < TT * TT; u += blockDim.x) {
        const int r = u / TT, c = u % TT, row = m0 + r, col = n0 + c;
        if (row < PO && col < PV) T[r][c] = src[((int64_t)K * PO + row) * lds + col];
    }
    __syncthreads();
    for (int u = threadIdx.x; u < TT * TT; u += blockDim.x) {
        const int r = u / TT, c = u % TT, row = n0 + r, col = m0 + c;
        if (row < PV && col < PO) dst[((int64_t)K * PV + row) * ldd + col] = T[c][r];
    }
}

// oovv_pk[K][p'][p] = <m km, n kn || e ke, f kf> for canonical (km, m, n) = p' and canonical
// (ke, e, f) = p of group K: the B operand of the W_mnij product (static).
__global__ void k_oovv_pack(Dims d, const int32_t *kc, PairTabs pt, const cd *oovv, uint16_t *out, bool c64) {
    const int N = d.N, no = d.no, nv = d.nv;
    const int nch = pt.PV / 8;
    const int64_t total = (int64_t)N * pt.PO * nch;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < total; x += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(x % nch);
        const int64_t row = x / nch;  // K * PO + p'
        const int K = (int)(row / pt.PO);
        const int pmn = pt.olist[row];
        cd v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int pef = pt.vlist[(int64_t)K * pt.PV + c * 8 + q];
            if (pmn < 0 || pef < 0) {
                v[q] = make_double2(0.0, 0.0);
                continue;
            }
            const int km = pmn / (no * no), mm = (pmn / no) % no, nn = pmn % no;
            const int ke = pef / (nv * nv), e = (pef / nv) % nv, f = pef % nv;
            const int kn = kcv(kc, N, K, 0, km);
            v[q] = oovv[blk3(N, km, kn, ke) * d.t2blk() + (((int64_t)mm * no + nn) * nv + e) * nv + f];
        }
        put_chunk(out, row * pt.PV + (int64_t)c * 8, v, c64);
    }
}

// Vt_pk[K][p'][p] = <ab||ef> + t_m^b <m kb, a ka||ef> - t_m^a <m ka, b kb||ef> for canonical
// (ka, a, b) = p' and (ke, e, f) = p.  The same workgroup layout as the full dressing (one
// workgroup per (ka, kb, ke, e), a thread per (b, f) running over a, <m kb, a ka||e f> in
// LDS, <m ka, b kb||e f> over m in registers), restricted to the blocks and elements that
// are canonical in both pairs: a quarter of the reads and writes of the full copy.  The
// grid covers only those blocks (pt.dblk), so the work is spread evenly over the XCDs.
// <m kb, a ka||e f> is staged in LDS (element type GT, GC elements) for as many a at a
// time as fit (all of them when o v^2 <= GC).  For n_occ <= OM and o v <= 2048.
// EX: exactly n_occ = OM, n_vir = 16 as constants (the branches on the orbital counts fold
// away, so the LDS reads of consecutive m are issued together).  For 8 < n_occ <= 32 the
// complex64 values are staged as read (GT = cf, 8192 of them in 64 KB): n_occ = 12 with
// n_vir = 24 takes one pass over a instead of four (3.6 -> 2.6 ms at N_k=8, 12 x 32; those
// kernels are limited to two waves per SIMD by their registers anyway).  For n_occ <= 8
// the smaller stage keeps three workgroups per CU, which measured faster than one pass.
template <int OM, bool EX = false, class GT = cd, int GC = 2048>
__global__ __launch_bounds__(256) void k_vvvv_dress_pack(SysDev s, PairTabs pt, const cd *t1, uint16_t *out,
                                                         int64_t ld, bool c64) {
    __shared__ GT G1[GC];
    __shared__ cd TA[OM * 64];
    const int N = s.d.N, no = EX ? OM : s.d.no, nv = EX ? 16 : s.d.nv, vv = nv * nv;
    const int64_t v3 = (int64_t)vv * nv, v4 = v3 * nv, ov3 = (int64_t)no * v3;
    const int64_t nblk = (int64_t)pt.ndblk * nv;
    const int64_t per = (nblk + 7) / 8;
    const int64_t L = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
    if (L >= nblk) return;
    const int e = (int)(L % nv);
    const int64_t blk = pt.dblk[L / nv];
    const int ke = (int)(blk % N), kb = (int)((blk / N) % N), ka = (int)(blk / ((int64_t)N * N));
    const int K = kcv(s.kc, N, ka, kb, 0);
    // the complex64 copy of ovvv: the t1 terms are rounded to bf16 pairs with <ab||ef> anyway
    const cf *g1b = s.ovvv_c + blk3(N, kb, ka, ke) * ov3 + (int64_t)e * nv;
    const cf *g2b = s.ovvv_c + blk3(N, ka, kb, ke) * ov3 + (int64_t)e * nv;
    const cd *ta = t1 + (int64_t)ka * no * nv, *tb = t1 + (int64_t)kb * no * nv;
    const cf *vb = s.vvvv_c + (L / nv) * v4 + (int64_t)e * nv;  // the kept blocks follow dblk
    const int32_t *vpos_ab = pt.vpos + ((int64_t)K * N + ka) * vv;
    const int32_t *vpos_ef = pt.vpos + ((int64_t)K * N + ke) * vv + e * nv;
    // a chunk of ac values of a: no * ac * nv <= GC and no * ac <= OM * 64
    const int ac = min(min(nv, GC / (no * nv)), OM * 64 / no);
    for (int a0 = 0; a0 < nv; a0 += ac) {
        const int na = min(ac, nv - a0), anv = na * nv;
        if (a0) __syncthreads();
        for (int x = threadIdx.x; x < no * anv; x += blockDim.x) {
            const int m = x / anv, af = x % anv;
            from_cd(to_cd(g1b[(int64_t)m * v3 + (int64_t)(a0 + af / nv) * vv + af % nv]), G1[x]);
        }
        for (int x = threadIdx.x; x < no * na; x += blockDim.x) TA[x] = ta[(x / na) * nv + a0 + x % na];
        __syncthreads();
        for (int bf = threadIdx.x; bf < vv; bf += blockDim.x) {
            const int b = bf / nv, f = bf % nv;
            const int pef = vpos_ef[f];
            if (pef < 0) continue;
            cd g2[OM], t1b[OM];
#pragma unroll
            for (int m = 0; m < OM; ++m) {
                g2[m] = m < no ? to_cd(g2b[(int64_t)m * v3 + (int64_t)b * vv + f]) : make_double2(0.0, 0.0);
                t1b[m] = m < no ? tb[m * nv + b] : make_double2(0.0, 0.0);
            }
            // eight a at a time: their pair positions and <ab||ef> loaded together, without
            // branches, before any is used (one memory round trip per eight instead of one each)
            for (int a1 = 0; a1 < na; a1 += 8) {
                int pabs[8];
                float vx[8], vy[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int a = a0 + min(a1 + u, na - 1);
                    pabs[u] = vpos_ab[a * nv + b];
                    const cf v = vb[(int64_t)a * v3 + (int64_t)b * vv + f];
                    vx[u] = v.x;
                    vy[u] = v.y;
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int a = a1 + u;
                    if (a >= na || pabs[u] < 0) continue;
                    cd acc = make_double2((double)vx[u], (double)vy[u]);
#pragma unroll
                    for (int m = 0; m < OM; ++m)
                        if (m < no) {
                            cfma(acc, t1b[m], to_cd(G1[(m * na + a) * nv + f]));
                            acc = csub(acc, cmul(TA[m * na + a], g2[m]));
                        }
                    put_elem(out, ((int64_t)K * pt.PV + pabs[u]) * ld + pef, acc, c64);
                }
            }
        }
    }
}

// Plain form for other sizes: a thread per 8 consecutive p of one p', every term from
// global memory.
__global__ void k_vvvv_dress_pack_plain(SysDev s, PairTabs pt, const cd *t1, uint16_t *out, int64_t ld, bool c64) {
    const int N = s.d.N, no = s.d.no, nv = s.d.nv, vv = nv * nv;
    const int64_t v3 = (int64_t)vv * nv, v4 = v3 * nv, ov3 = (int64_t)no * v3;
    const int nch = pt.PV / 8;
    const int64_t total = (int64_t)N * pt.PV * nch;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < total; x += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(x % nch);
        const int64_t row = x / nch;  // K * PV + p'
        const int K = (int)(row / pt.PV);
        const int pab = pt.vlist[row];
        cd v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int pef = pt.vlist[(int64_t)K * pt.PV + c * 8 + q];
            v[q] = make_double2(0.0, 0.0);
            if (pab < 0 || pef < 0) continue;
            const int ka = pab / vv, a = (pab / nv) % nv, b = pab % nv;
            const int ke = pef / vv, e = (pef / nv) % nv, f = pef % nv;
            const int kb = kcv(s.kc, N, K, 0, ka);
            // (ka, kb, ke) is a kept block of <ab||ef>: ka <= kb and ke <= kf for canonical pairs
            const int64_t vk = s.vblk[blk3(N, ka, kb, ke)];
            cd acc = to_cd(s.vvvv_c[vk * v4 + (((int64_t)a * nv + b) * nv + e) * nv + f]);
            const cf *g1 = s.ovvv_c + blk3(N, kb, ka, ke) * ov3 + ((int64_t)a * nv + e) * nv + f;
            const cf *g2 = s.ovvv_c + blk3(N, ka, kb, ke) * ov3 + ((int64_t)b * nv + e) * nv + f;
            for (int m = 0; m < no; ++m) {
                cfma(acc, t1[((int64_t)kb * no + m) * nv + b], to_cd(g1[(int64_t)m * v3]));
                acc = csub(acc, cmul(t1[((int64_t)ka * no + m) * nv + a], to_cd(g2[(int64_t)m * v3])));
            }
            v[q] = acc;
        }
        put_chunk(out, row * ld + (int64_t)c * 8, v, c64);
    }
}

static dim3 pack_grid(int64_t threads) {
    int64_t b = (threads + 255) / 256;
    if (b > (1 << 20)) b = 1 << 20;
    return dim3((unsigned)(b < 1 ? 1 : b));
}

bool dress_pack_ok(const Dims &d) { return d.no <= 32 && (int64_t)d.no * d.nv <= 2048; }

void launch_tau_pack(const Dims &d, const int32_t *kc, const PairTabs &pt, const cd *t1, const cd *t2,
                     uint16_t *tau_pk, int64_t ld_tau, uint16_t *tauT_pk, int64_t ld_tauT, bool c64, hipStream_t st) {
    const int64_t N = d.N;
    const dim3 g = pack_grid(N * pt.PO * pt.PV);
    if (d.no == 8 && d.nv == 16)
        hipLaunchKernelGGL(k_tau_pack<true>, g, dim3(256), 0, st, d, kc, pt, t1, t2, tau_pk, ld_tau, c64);
    else
        hipLaunchKernelGGL(k_tau_pack<false>, g, dim3(256), 0, st, d, kc, pt, t1, t2, tau_pk, ld_tau, c64);
    CK_CHECK(hipGetLastError());
    const dim3 gt((unsigned)((pt.PV + TT - 1) / TT), (unsigned)((pt.PO + TT - 1) / TT), (unsigned)N);
    if (c64)
        hipLaunchKernelGGL(k_tau_transpose_c64, gt, dim3(256), 0, st, pt.PO, pt.PV, (const uint2 *)tau_pk, ld_tau,
                           (uint2 *)tauT_pk, ld_tauT);
    else
        hipLaunchKernelGGL(k_tau_transpose, gt, dim3(256), 0, st, pt.PO, pt.PV, tau_pk, ld_tau, tauT_pk, ld_tauT);
    CK_CHECK(hipGetLastError());
}

void launch_oovv_pack(const Dims &d, const int32_t *kc, const PairTabs &pt, const cd *oovv, uint16_t *out, bool c64,
                      hipStream_t st) {
    const int64_t N = d.N;
    hipLaunchKernelGGL(k_oovv_pack, pack_grid(N * pt.PO * (pt.PV / 8)), dim3(256), 0, st, d, kc, pt, oovv, out, c64);
    CK_CHECK(hipGetLastError());
}

void launch_vvvv_dress_pack(const SysDev &s, const PairTabs &pt, const cd *t1, uint16_t *out, int64_t ld, bool c64,
                            hipStream_t st) {
    const int64_t N = s.d.N, nv = s.d.nv;
    const int64_t n = (int64_t)pt.ndblk * nv;
    const dim3 grid((unsigned)((n + 7) / 8 * 8));
    if (!dress_pack_ok(s.d))
        hipLaunchKernelGGL(k_vvvv_dress_pack_plain, pack_grid(N * pt.PV * (pt.PV / 8)), dim3(256), 0, st, s, pt, t1,
                           out, ld, c64);
    else if (s.d.no == 8 && nv == 16)
        hipLaunchKernelGGL((k_vvvv_dress_pack<8, true>), grid, dim3(256), 0, st, s, pt, t1, out, ld, c64);
    else if (s.d.no <= 8)
        hipLaunchKernelGGL((k_vvvv_dress_pack<8>), grid, dim3(256), 0, st, s, pt, t1, out, ld, c64);
    else if (s.d.no <= 16)
        hipLaunchKernelGGL((k_vvvv_dress_pack<16, false, cf, 8192>), grid, dim3(256), 0, st, s, pt, t1, out, ld, c64);
    else
        hipLaunchKernelGGL((k_vvvv_dress_pack<32, false, cf, 8192>), grid, dim3(256), 0, st, s, pt, t1, out, ld, c64);
    CK_CHECK(hipGetLastError());
}

// ------------------------------------------------------------------ R2 assembly
// r2 = <ab||ij>* + P(ij)P(ab) X + L (the driver term from the complex64 copy of <ij||ab>),
// with L the ladders' packed result Lp[K][p'][p]
// (canonical (ki, i, j) = p', canonical (ka, a, b) = p) expanded by antisymmetry:
// L(ij, ab) = s_ij s_ab Lp[canonical ij][canonical ab], s = -1 for a pair in the
// non-canonical order, 0 for a pair of two equal members.
//
// The four R2 blocks B1 = (ki, kj, ka; i, j), B2 = (kj, ki, ka; j, i), B3 = (ki, kj, kb; i, j)
// and B4 = (kj, ki, kb; j, i) use the same four v x v slabs of X,
//   Xa = X(ki, kj, ka; i, j), Xb = X(kj, ki, ka; j, i), Xc = X(ki, kj, kb; i, j),
//   Xd = X(kj, ki, kb; j, i),
// each straight and transposed, so one workgroup takes the whole orbit: the slabs are read
// once into LDS and every member is written with the two-pair formula
//   B(a, b) = (x1 + x4) - (x2 + x3),  x1 = own slab (a, b), x2 = the ij partner's (a, b),
//   x3 = the ab partner's (b, a), x4 = the (ij, ab) partner's (b, a),
// exactly as a workgroup per block would (the members are exact negatives and transposes
// of each other).  Workgroups run over the orbit representatives pt.ablk (ki <= kj,
// ka <= kb) times the (i, j) with i <= j when ki == kj; members that coincide with the
// representative (ki == kj and i == j, or ka == kb) are not written twice.
constexpr int ASMP_VMAX = 31;  // four padded slabs within 64 KB of dynamic LDS

// The packed ladder value of the virtual pair (x at kx, y at ky) in the row Lrow: the stored
// canonical value, its negative for the exchanged pair, zero on the diagonal.  Branch free
// (the address is selected, the load always made), so that the loads of an element are in
// flight together.
__device__ inline cd asm_lab(const cd *Lrow, const int32_t *vposK, int vv, int nv, int kx, int x, int ky, int y) {
    const bool fwd = kx < ky || (kx == ky && x < y), diag = kx == ky && x == y;
    const int pos = vposK[fwd ? (int64_t)kx * vv + x * nv + y : (int64_t)ky * vv + y * nv + x];
    const cd l = Lrow[diag ? 0 : pos];
    return diag ? make_double2(0.0, 0.0) : fwd ? l : make_double2(-l.x, -l.y);
}

// Sum of |x|^2 over the workgroup (256 threads), in a fixed order; the result is valid in
// thread 0.
__device__ inline double asm_block_sum(double v, double *sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    return sh[0];
}

// npart[blockIdx.x] receives the sum of |r2|^2 over the elements this workgroup writes (0
// for a workgroup without an orbit), so that the residual norm needs no second pass over R2.
__global__ __launch_bounds__(256) void k_assemble_r2_pack(SysDev s, PairTabs pt, const cd *X, const cd *Lp, cf *r2,
                                                          double *npart) {
    extern __shared__ cd XS[];  // four slabs, rows padded to nv + 1 (LDS form only)
    __shared__ double NS[256];
    const int N = s.d.N, no = s.d.no, nv = s.d.nv, vv = nv * nv, vp = nv + 1;
    const int64_t ov = (int64_t)no * nv, ov2 = ov * ov, bs = s.d.t2blk();
    const int64_t nblk = (int64_t)pt.nablk * no * no;
    const int64_t per = (nblk + 7) / 8;
    const int64_t L = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
    const int64_t Lc = L < nblk ? L : 0;
    const int j = (int)(Lc % no), i = (int)((Lc / no) % no);
    const int blk = pt.ablk[Lc / ((int64_t)no * no)];
    const int ka = blk % N, kj = (blk / N) % N, ki = blk / (N * N);
    if (L >= nblk || (ki == kj && i > j)) {
        if (threadIdx.x == 0) npart[blockIdx.x] = 0.0;
        return;
    }
    const int kb = kcv(s.kc, N, ki, kj, ka), K = kcv(s.kc, N, ki, kj, 0);
    const bool own_ij = ki == kj && i == j, own_ab = ka == kb;
    // slab (x at k1, y at k2; a-slot momentum k3): X[q = k3 - k1][k1][k2](x, ., y, .)
    auto slab = [&](int k1, int k2, int k3, int x, int y) {
        const int q = kcv(s.kc, N, k3, 0, k1);
        return X + (((int64_t)q * N + k1) * N + k2) * ov2 + (int64_t)x * nv * ov + (int64_t)y * nv;
    };
    const cd *sa = slab(ki, kj, ka, i, j), *sb = slab(kj, ki, ka, j, i);
    const cd *sc = slab(ki, kj, kb, i, j), *sd = slab(kj, ki, kb, j, i);
    const bool lds = nv <= ASMP_VMAX;
    cd *Xa = XS, *Xb = XS + nv * vp, *Xc = XS + 2 * nv * vp, *Xd = XS + 3 * nv * vp;
    if (lds) {
        for (int e = threadIdx.x; e < vv; e += blockDim.x) {
            const int a = e / nv, b = e % nv;
            const int64_t g = (int64_t)a * ov + b;
            Xa[a * vp + b] = sa[g];
            Xb[a * vp + b] = sb[g];
            Xc[a * vp + b] = sc[g];
            Xd[a * vp + b] = sd[g];
        }
        __syncthreads();
    }
    auto at = [&](const cd *sm, const cd *sg, int a, int b) {
        return lds ? sm[a * vp + b] : sg[(int64_t)a * ov + b];
    };
    const int po = own_ij ? -1 : pt.opos[((int64_t)K * N + ki) * no * no + i * no + j];
    const cd *Lrow = Lp + ((int64_t)K * pt.PO + (po < 0 ? 0 : po)) * pt.PV;
    const int32_t *vposK = pt.vpos + (int64_t)K * N * vv;
    const int64_t o1 = blk3(N, ki, kj, ka) * bs + ((int64_t)i * no + j) * vv;
    const int64_t o2 = blk3(N, kj, ki, ka) * bs + ((int64_t)j * no + i) * vv;
    const int64_t o3 = blk3(N, ki, kj, kb) * bs + ((int64_t)i * no + j) * vv;
    const int64_t o4 = blk3(N, kj, ki, kb) * bs + ((int64_t)j * no + i) * vv;
    double nsq = 0.0;
    auto put = [&](int64_t o, cd v) {  // stored in complex64; the norm is taken from the stored value
        cf c;
        from_cd(v, c);
        r2[o] = c;
        const cd w = to_cd(c);
        nsq = fma(w.x, w.x, fma(w.y, w.y, nsq));
    };
    for (int e = threadIdx.x; e < vv; e += blockDim.x) {
        const int a = e / nv, b = e % nv;
        // every global load of the element first and without branches (members that do not
        // exist re-read the first one's integral, a cache hit), one round trip together
        const cf g1 = s.oovv_c[o1 + e], g2 = s.oovv_c[(own_ij ? o1 : o2) + e];
        const cf g3 = s.oovv_c[(own_ab ? o1 : o3) + e], g4 = s.oovv_c[(own_ab || own_ij ? o1 : o4) + e];
        const cd la = asm_lab(Lrow, vposK, vv, nv, ka, a, kb, b), lb = asm_lab(Lrow, vposK, vv, nv, kb, a, ka, b);
        const cd l1 = po < 0 ? make_double2(0.0, 0.0) : la;
        {  // B1 and B2
            const cd x1 = at(Xa, sa, a, b), x2 = at(Xb, sb, a, b), x3 = at(Xc, sc, b, a), x4 = at(Xd, sd, b, a);
            const cd d1 = cconj(to_cd(g1));
            const cd p1 = make_double2((x1.x + x4.x) - (x2.x + x3.x), (x1.y + x4.y) - (x2.y + x3.y));
            put(o1 + e, make_double2((d1.x + p1.x) + l1.x, (d1.y + p1.y) + l1.y));
            if (!own_ij) {
                const cd d2 = cconj(to_cd(g2));
                const cd p2 = make_double2((x2.x + x3.x) - (x1.x + x4.x), (x2.y + x3.y) - (x1.y + x4.y));
                put(o2 + e, make_double2((d2.x + p2.x) - l1.x, (d2.y + p2.y) - l1.y));
            }
        }
        if (!own_ab) {  // B3 and B4: the a slot at kb
            const cd l3 = po < 0 ? make_double2(0.0, 0.0) : lb;
            const cd x1 = at(Xc, sc, a, b), x2 = at(Xd, sd, a, b), x3 = at(Xa, sa, b, a), x4 = at(Xb, sb, b, a);
            const cd d3 = cconj(to_cd(g3));
            const cd p3 = make_double2((x1.x + x4.x) - (x2.x + x3.x), (x1.y + x4.y) - (x2.y + x3.y));
            put(o3 + e, make_double2((d3.x + p3.x) + l3.x, (d3.y + p3.y) + l3.y));
            if (!own_ij) {
                const cd d4 = cconj(to_cd(g4));
                const cd p4 = make_double2((x2.x + x3.x) - (x1.x + x4.x), (x2.y + x3.y) - (x1.y + x4.y));
                put(o4 + e, make_double2((d4.x + p4.x) - l3.x, (d4.y + p4.y) - l3.y));
            }
        }
    }
    const double tot = asm_block_sum(nsq, NS);
    if (threadIdx.x == 0) npart[blockIdx.x] = tot;
}

// out = sum_b npart[b] + sum |r1|^2: one workgroup of 1024 threads, each with four
// independent partial sums over a fixed strided subset (so that four loads are in flight),
// combined in a fixed order and then by a fixed LDS tree
__global__ __launch_bounds__(1024) void k_norm_final(const double *npart, int64_t nb, const cd *r1, int64_t n1,
                                                     double *out) {
    __shared__ double NS[1024];
    const int t = threadIdx.x;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t b0 = t; b0 < nb; b0 += 4 * 1024) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t b = b0 + (int64_t)u * 1024;
            if (b < nb) v[u] += npart[b];
        }
    }
    for (int64_t x = t; x < n1; x += 1024) v[0] = fma(r1[x].x, r1[x].x, fma(r1[x].y, r1[x].y, v[0]));
    NS[t] = (v[0] + v[1]) + (v[2] + v[3]);
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (t < w) NS[t] += NS[t + w];
        __syncthreads();
    }
    if (t == 0) out[0] = NS[0];
}

int64_t assemble_pack_blocks(const Dims &d, const PairTabs &pt) {
    const int64_t n = (int64_t)pt.nablk * d.no * d.no;
    return (n + 7) / 8 * 8;
}

void launch_norm_pack(const Dims &d, const PairTabs &pt, const double *npart, const cd *r1, double *out,
                      hipStream_t st) {
    hipLaunchKernelGGL(k_norm_final, dim3(1), dim3(1024), 0, st, npart, assemble_pack_blocks(d, pt), r1, d.t1(), out);
    CK_CHECK(hipGetLastError());
}

void launch_assemble_r2_pack(const SysDev &s, const PairTabs &pt, const cd *X, const cd *Lp, cf *r2, double *npart,
                             hipStream_t st) {
    const int64_t nv = s.d.nv;
    const int64_t nb = assemble_pack_blocks(s.d, pt);
    if (nb == 0) return;
    const size_t lds = nv <= ASMP_VMAX ? (size_t)4 * nv * (nv + 1) * sizeof(cd) : 0;
    hipLaunchKernelGGL(k_assemble_r2_pack, dim3((unsigned)nb), dim3(256), lds, st, s, pt, X, Lp, r2, npart);
    CK_CHECK(hipGetLastError());
}

// ------------------------------------------------------------------ DIIS extrapolation
// t <- sum_j c_j src_j for the mixed path, split in two passes over the (t1 | t2) vector:
// the t1 part (with the f_ia t_i^a term of the correlation energy), then the t2 part, which
// (k_lincomb_t2_pack, from the packed history below) also writes the operand copy of t2 that
// the next residual's products read and the t2 terms
// of the energy at the new amplitudes (they need the new t1, hence the order).  The energy
// is 1/4 <ij||ab> t_ij^ab + 1/2 <ij||ab> t_i^a t_j^b (k_a = k_i) summed over every stored
// element, plus sum f_ia t_i^a, exactly as the stand-alone energy pass (both with the
// complex64 copy of <ij||ab>).

__device__ inline void blk_sum2(double &x, double &y, double (*sh)[256]) {
    const int t = threadIdx.x;
    sh[0][t] = x;
    sh[1][t] = y;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) {
            sh[0][t] += sh[0][t + w];
            sh[1][t] += sh[1][t + w];
        }
        __syncthreads();
    }
    x = sh[0][0];
    y = sh[1][0];
}

constexpr int LINPACK_VMAX = 48;  // largest n_vir whose v x (v + 1) slab the extrapolation keeps in LDS

template <class ET>
struct ErrPack {
    ET *p[16];
};
struct HistPackD {
    cd *p[16];
};
constexpr int UPD_PACK_BLOCKS = UPD_BLOCKS;  // the partials buffer is sized for UPD_BLOCKS

// sixteen running sums over the workgroup (fixed order); valid in v after the call
__device__ inline void blk_sum16(double (&v)[16], double (*sh)[256]) {
    const int t = threadIdx.x;
#pragma unroll
    for (int j = 0; j < 16; ++j) sh[j][t] = v[j];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w)
#pragma unroll
            for (int j = 0; j < 16; ++j) sh[j][t] += sh[j][t + w];
        __syncthreads();
    }
#pragma unroll
    for (int j = 0; j < 16; ++j) v[j] = sh[j][0];
}

__global__ __launch_bounds__(256) void k_lincomb_t1(SysDev s, LincombArgs L, DiisDev dd, Gate gate, cd *t, double *ep1) {
    if (!gate.open()) return;
    const int m = dd.state[1];
    __shared__ double sh[2][256];
    const int no = s.d.no, nv = s.d.nv, n = no + nv;
    const int64_t n1 = s.d.t1();
    double er = 0.0, ei = 0.0;
    for (int64_t idx = threadIdx.x; idx < n1; idx += 256) {
        cd acc = make_double2(0.0, 0.0);
        for (int j = 0; j < m; ++j) {
            const cd x = L.src[j][idx];
            const double c = dd.coef[j];
            acc.x = fma(c, x.x, acc.x);
            acc.y = fma(c, x.y, acc.y);
        }
        t[idx] = acc;
        const int a = (int)(idx % nv), i = (int)((idx / nv) % no), k = (int)(idx / ((int64_t)no * nv));
        const cd p = cmul(s.fock[((int64_t)k * n + i) * n + no + a], acc);
        er += p.x;
        ei += p.y;
    }
    blk_sum2(er, ei, sh);
    if (threadIdx.x == 0 && ep1) {
        ep1[0] = er;
        ep1[1] = ei;
    }
}

// out[0..1] = ep1 + sum_b ep2, in a fixed order: one workgroup of 1024 threads, each with
// four independent partial sums over a fixed strided subset (so that four loads of each
// part are in flight), combined in a fixed order and then by a fixed LDS tree
__global__ __launch_bounds__(1024) void k_energy_final(const double *ep1, const double *ep2, int nb, double *out) {
    __shared__ double sh[2][1024];
    const int t = threadIdx.x;
    double vr[4] = {0.0, 0.0, 0.0, 0.0}, vi[4] = {0.0, 0.0, 0.0, 0.0};
    for (int b0 = t; b0 < nb; b0 += 4 * 1024) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int b = b0 + u * 1024;
            if (b < nb) {
                vr[u] += ep2[b];
                vi[u] += ep2[nb + b];
            }
        }
    }
    sh[0][t] = (vr[0] + vr[1]) + (vr[2] + vr[3]);
    sh[1][t] = (vi[0] + vi[1]) + (vi[2] + vi[3]);
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if (t < w) {
            sh[0][t] += sh[0][t + w];
            sh[1][t] += sh[1][t + w];
        }
        __syncthreads();
    }
    if (t == 0) {
        out[0] = ep1[0] + sh[0][0];
        out[1] = ep1[1] + sh[1][0];
    }
}

// ------------------------------------------------------------------ packed DIIS history
// The DIIS vectors hold t1 in full and t2 only on the representative block of each
// antisymmetry orbit (pt.ablk: ki <= kj, ka <= kb; the whole o^2 v^2 block):
// packed element (r, x) is t2[ablk[r]][x].  Every orbit member is +- a representative
// element (t_ij^ab = -t_ji^ab = -t_ij^ba with the momenta), so an overlap over the full
// vector is the packed overlap with weight w(r) = (ki < kj ? 2 : 1) (ka < kb ? 2 : 1) on
// block r: the coefficients are the full ones, from about a quarter of the bytes.
__device__ inline double pack_weight(int N, int blk, const int32_t *kc) {
    const int ka = blk % N, kj = (blk / N) % N, ki = blk / (N * N);
    const int kb = kc[blk];
    return (ki < kj ? 2.0 : 1.0) * (ka < kb ? 2.0 : 1.0);
}

// RT: element type of R2 (complex64 on the mixed path), ET: of the stored error vectors
template <bool EX, class RT, class ET>
__global__ __launch_bounds__(256) void k_update_diis_pack(SysDev s, PairTabs pt, const cd *t, const cd *r1, const RT *r2,
                                                          ErrPack<ET> y, HistPackD hp, DiisDev dd, Gate gate,
                                                          double *partials) {
    if (!gate.open()) return;
    using EV = decltype(ET{}.x);
    const int self = dd.state[0], m = min(dd.state[1] + 1, dd.m);
    ET *err = y.p[self];
    cd *hist = hp.p[self];
    __shared__ double sh[16][256];
    const int N = s.d.N, no = EX ? 8 : s.d.no, nv = EX ? 16 : s.d.nv;
    const int64_t n1 = (int64_t)N * no * nv, bs = (int64_t)no * no * nv * nv;
    const int vv = nv * nv;
    double v[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) v[j] = 0.0;
    // one element: packed position idx, position in the full (t1 | t2) vector, denominator,
    // overlap weight
    auto elem = [&](int64_t idx, int64_t full, double D, double w) {
        const cd rv = idx < n1 ? r1[idx] : to_cd(r2[full - n1]);
        const cd tv = t[full];
        // the stored error vectors of this element, loaded before any is used and without
        // branches (a load under a branch is waited for inside it), so that they take one
        // memory round trip for the element instead of one each: the first eight
        // unconditionally, those beyond the space in use re-reading vector 0 (a cache hit);
        // larger spaces load the rest one by one
        EV bx[16], by[16];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const ET b = (j < m ? y.p[j] : y.p[0])[idx];
            bx[j] = b.x;
            by[j] = b.y;
        }
#pragma unroll
        for (int j = 8; j < 16; ++j) {
            bx[j] = EV(0);
            by[j] = EV(0);
            if (j < m) {
                const ET b = y.p[j][idx];
                bx[j] = b.x;
                by[j] = b.y;
            }
        }
        const double iD = 1.0 / D;
        const cd e = make_double2(rv.x * iD, rv.y * iD);
        hist[idx] = cadd(tv, e);
        ET es;
        from_cd(e, es);
        const cd ed = to_cd(es);
#pragma unroll
        for (int j = 0; j < 16; ++j)
            if (j < m) {
                const cd b = j == self ? ed : make_double2((double)bx[j], (double)by[j]);
                v[j] = fma(w, fma(ed.x, b.x, ed.y * b.y), v[j]);
            }
        err[idx] = es;
    };
    // t1: spread over the grid
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n1; idx += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)idx;
        const int a = x % nv, i = (x / nv) % no, k = x / (no * nv);
        elem(idx, idx, s.eo[k * no + i] - s.ev[k * nv + a], 1.0);
    }
    // t2: (representative block, i, j) slabs of v^2 elements, a workgroup pass covering one
    // slab (v^2 >= 256: its block, momenta and weight are the same for the whole workgroup) or
    // 256 / v^2 consecutive slabs, so that the table look-ups are made once per slab
    const int64_t nslab = (int64_t)pt.nablk * no * no;
    const int spw = vv >= 256 ? 1 : 256 / vv;
    const int lane_slab = vv >= 256 ? 0 : (int)threadIdx.x / vv;
    const int x0 = vv >= 256 ? (int)threadIdx.x : (int)threadIdx.x % vv, xs = vv >= 256 ? 256 : vv;
    for (int64_t s0 = (int64_t)blockIdx.x * spw; s0 < nslab; s0 += (int64_t)gridDim.x * spw) {
        const int64_t sl = s0 + lane_slab;
        if (lane_slab >= spw || sl >= nslab) continue;
        const int64_t r = sl / (no * no);
        const int ij = (int)(sl - r * no * no), i = ij / no, j = ij % no;
        const int blk = pt.ablk[r];
        const int ka = blk % N, kj = (blk / N) % N, ki = blk / (N * N);
        const int kb = s.kc[blk];
        const double w = pack_weight(N, blk, s.kc);
        const double Dij = s.eo[ki * no + i] + s.eo[kj * no + j];
        for (int x = x0; x < vv; x += xs) {
            const int a = x / nv, b = x % nv;
            const int64_t xb = (int64_t)ij * vv + x;
            elem(n1 + r * bs + xb, n1 + (int64_t)blk * bs + xb, Dij - s.ev[ka * nv + a] - s.ev[kb * nv + b], w);
        }
    }
    blk_sum16(v, sh);
    if (threadIdx.x == 0)
        for (int j = 0; j < m; ++j) partials[(int64_t)j * UPD_PACK_BLOCKS + blockIdx.x] = v[j];
}

// t2 part of the extrapolation from packed history: a workgroup per (representative block,
// i, j) (i <= j when ki == kj) forms the v x v slab sum_j c_j hist_j in LDS and writes the
// orbit's members, t(ki,kj,ka; i,j) = L, t(kj,ki,ka; j,i) = -L, t(ki,kj,kb; i,j) = -L^T,
// t(kj,ki,kb; j,i) = L^T (members that coincide with another are written once), each also
// into the operand storage of the ring family (sp) and into the energy partial sums
// (1/4 <ij||ab> t_ij^ab + 1/2 <ij||ab> t_i^a t_j^b, k_a = k_i, per written element).
__global__ __launch_bounds__(256) void k_lincomb_t2_pack(SysDev s, PairTabs pt, LincombArgs L, DiisDev dd, Gate gate,
                                                         cd *t, uint16_t *sp, bool c64, double *ep2) {
    if (!gate.open()) return;
    const int m = dd.state[1];
    extern __shared__ cd SL[];  // v x (v + 1) (LDS form, n_vir <= LINPACK_VMAX)
    __shared__ double sh[2][256];
    const int N = s.d.N, no = s.d.no, nv = s.d.nv, vv = nv * nv, vp = nv + 1;
    const bool lds = nv <= LINPACK_VMAX;
    const int64_t n1 = s.d.t1(), bs = s.d.t2blk();
    const int64_t nblk = (int64_t)pt.nablk * no * no;
    const int64_t L0 = blockIdx.x;
    const int j = (int)(L0 % no), i = (int)((L0 / no) % no);
    const int64_t r = L0 / ((int64_t)no * no);
    double er = 0.0, ei = 0.0;
    const int blk = r < pt.nablk ? pt.ablk[r] : 0;
    const int ka = blk % N, kj = (blk / N) % N, ki = blk / (N * N);
    const bool live = L0 < nblk && !(ki == kj && i > j);
    if (live) {
        const int kb = kcv(s.kc, N, ki, kj, ka);
        const int64_t src = n1 + r * bs + ((int64_t)i * no + j) * vv;
        // sum_q c_q hist_q at e: the first eight vectors loaded without branches before any is
        // used (those beyond the space in use re-read vector 0 and take coefficient 0), so they
        // take one memory round trip; larger spaces add the rest one by one
        auto comb = [&](int e) {
            double xr[8], xi[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const cd x = (q < m ? L.src[q] : L.src[0])[src + e];
                xr[q] = x.x;
                xi[q] = x.y;
            }
            cd acc = make_double2(0.0, 0.0);
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const double c = q < m ? dd.coef[q] : 0.0;
                acc.x = fma(c, xr[q], acc.x);
                acc.y = fma(c, xi[q], acc.y);
            }
            for (int q = 8; q < m; ++q) {
                const cd x = L.src[q][src + e];
                const double c = dd.coef[q];
                acc.x = fma(c, x.x, acc.x);
                acc.y = fma(c, x.y, acc.y);
            }
            return acc;
        };
        if (lds) {
            for (int e = threadIdx.x; e < vv; e += blockDim.x) SL[(e / nv) * vp + e % nv] = comb(e);
            __syncthreads();
        }
        const cd *t1 = t;  // the new t1 (written by k_lincomb_t1 before this pass)
        // one member: block (k1, k2, k3) with the pair (x at k1, y at k2) and a-slot momentum k3
        auto put = [&](int k1, int k2, int k3, int x, int y, int a, int b, cd v) {
            const int64_t o = blk3(N, k1, k2, k3) * bs + ((int64_t)x * no + y) * vv + (int64_t)a * nv + b;
            t[n1 + o] = v;
            if (!ep2) return;  // the FP64 path: no operand copy, the energy by its own pass
            put_elem(sp, o, v, c64);
            cd wv = cscale(v, 0.25);
            if (k3 == k1)
                wv = cadd(wv, cscale(cmul(t1[((int64_t)k1 * no + x) * nv + a], t1[((int64_t)k2 * no + y) * nv + b]), 0.5));
            const cd p = cmul(to_cd(s.oovv_c[o]), wv);
            er += p.x;
            ei += p.y;
        };
        const bool own_ij = ki == kj, own_ab = ka == kb;
        for (int e = threadIdx.x; e < vv; e += blockDim.x) {
            const int a = e / nv, b = e % nv;
            const cd l = lds ? SL[a * vp + b] : comb(e), lt = lds ? SL[b * vp + a] : comb(b * nv + a);
            put(ki, kj, ka, i, j, a, b, l);
            if (!own_ij || i != j) {
                if (!own_ij) put(kj, ki, ka, j, i, a, b, make_double2(-l.x, -l.y));
                else put(ki, ki, ka, j, i, a, b, make_double2(-l.x, -l.y));  // the (j, i) slab of the same block
            }
            if (!own_ab) {
                put(ki, kj, kb, i, j, a, b, make_double2(-lt.x, -lt.y));
                if (!own_ij) put(kj, ki, kb, j, i, a, b, lt);
                else if (i != j) put(ki, ki, kb, j, i, a, b, lt);
            }
        }
    }
    if (!ep2) return;
    blk_sum2(er, ei, sh);
    if (threadIdx.x == 0) {
        ep2[blockIdx.x] = er;
        ep2[gridDim.x + blockIdx.x] = ei;
    }
}

int64_t packed_len(const Dims &d, const PairTabs &pt) { return d.t1() + (int64_t)pt.nablk * d.t2blk(); }

template <class RT, class ET>
static void update_diis_pack(const SysDev &s, const PairTabs &pt, const cd *t, const cd *r1, const RT *r2,
                             ET *const *err, cd *const *hist, const DiisDev &dd, Gate gate, double *partials,
                             hipStream_t st) {
    ErrPack<ET> pk{};
    HistPackD hp{};
    for (int j = 0; j < dd.m; ++j) {
        pk.p[j] = err[j];
        hp.p[j] = hist[j];
    }
    if (s.d.no == 8 && s.d.nv == 16)
        hipLaunchKernelGGL((k_update_diis_pack<true, RT, ET>), dim3(UPD_PACK_BLOCKS), dim3(256), 0, st, s, pt, t, r1,
                           r2, pk, hp, dd, gate, partials);
    else
        hipLaunchKernelGGL((k_update_diis_pack<false, RT, ET>), dim3(UPD_PACK_BLOCKS), dim3(256), 0, st, s, pt, t, r1,
                           r2, pk, hp, dd, gate, partials);
    CK_CHECK(hipGetLastError());
    launch_diis_solve(dd, gate, partials, UPD_PACK_BLOCKS, st);
}
void launch_update_diis_pack(const SysDev &s, const PairTabs &pt, const cd *t, const cd *r1, const cf *r2,
                             cf *const *err, cd *const *hist, const DiisDev &dd, Gate gate, double *partials,
                             hipStream_t st) {
    update_diis_pack(s, pt, t, r1, r2, err, hist, dd, gate, partials, st);
}
void launch_update_diis_pack(const SysDev &s, const PairTabs &pt, const cd *t, const cd *r1, const cd *r2,
                             cd *const *err, cd *const *hist, const DiisDev &dd, Gate gate, double *partials,
                             hipStream_t st) {
    update_diis_pack(s, pt, t, r1, r2, err, hist, dd, gate, partials, st);
}

int64_t lincomb_pack_blocks(const Dims &d, const PairTabs &pt) { return std::max<int64_t>(1, (int64_t)pt.nablk * d.no * d.no); }

void launch_lincomb_packed(const SysDev &s, const PairTabs &pt, const cd *const *src, const DiisDev &dd, Gate gate,
                           cd *t, uint16_t *sp, bool c64, double *epart, hipStream_t st) {
    LincombArgs L{};
    for (int j = 0; j < dd.m; ++j) L.src[j] = src[j];
    hipLaunchKernelGGL(k_lincomb_t1, dim3(1), dim3(256), 0, st, s, L, dd, gate, t, epart);
    CK_CHECK(hipGetLastError());
    const int64_t nb = lincomb_pack_blocks(s.d, pt);
    const size_t lds = s.d.nv <= LINPACK_VMAX ? (size_t)s.d.nv * (s.d.nv + 1) * sizeof(cd) : 0;
    hipLaunchKernelGGL(k_lincomb_t2_pack, dim3((unsigned)nb), dim3(256), lds, st, s, pt, L, dd, gate, t, sp, c64,
                       epart ? epart + 2 : nullptr);
    CK_CHECK(hipGetLastError());
}

void launch_energy_packed(const Dims &d, const PairTabs &pt, const double *epart, double *out, hipStream_t st) {
    hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(1024), 0, st, epart, epart + 2, (int)lincomb_pack_blocks(d, pt), out);
    CK_CHECK(hipGetLastError());
}


}  // namespace ck
