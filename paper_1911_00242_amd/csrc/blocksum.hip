// Register-tiled block sums of the F intermediates and of the T1 residual for
// n_occ <= 16, n_vir <= 32 outside the 8 x 16 tile (the shapes of the larger batched
// systems).  Per momentum block (p, q, r) with fourth momentum kb, each of the four sums
// is, for every n, a small product over LDS-staged slabs,
//   out(row, col) += sum_k X(row, k) Y(col, k),
//   Foo (m, i): X = <mn||ef>,               Y = tau-tilde(i,n,e,f),  k = (e, f)
//   Fvv (a, e): X = tau-tilde(m,n,a,f),     Y = <mn||ef>,            k = (m, f)
//   P1a (i, a): X = t2(i,n,e,f),            Y = <n q, a p||e r, f>,  k = (e, f)
//   P1b (i, a): X = <m p, n q||i r, f>,     Y = t2(m,n,a,f),         k = (m, f)
// (the tau-tilde sums of F_mi and F_ae and the two t2-integral sums of the T1 equation,
// Sec. 2; the results go to the same partial arrays, with the same factors, as the other
// forms of these sums).  A workgroup takes one block and one range of its slabs (n, chunk
// of e or of m); the slab is staged in LDS with the next one prefetched into registers
// (loaded as stored, without arithmetic between the loads), and each thread accumulates a
// 4 x 4 tile of outputs over its share of k, so eight LDS reads feed sixteen complex
// multiply-adds.  The tiles are laid over the actual n_occ and n_vir, so no work is spent
// on padding; threads per tile = 256 / tiles.  The partial sums of a tile are combined in
// a fixed order, so results do not depend on the launch.
#include <type_traits>

#include "terms.h"

namespace ck {

namespace {

// n / d for n < 2^16, 1 <= d < 2^16 by one multiply: with m = ceil(2^32 / d) the error of
// n m / 2^32 against n / d is below n / 2^32 < 1 / d, which cannot reach the next integer.
struct FastDiv {
    uint64_t m;
    __device__ explicit FastDiv(uint32_t d) : m((0x100000000ull + d - 1) / d) {}
    __device__ uint32_t operator()(uint32_t n) const { return (uint32_t)(((uint64_t)n * m) >> 32); }
};

template <int PASS, int OM, int VM>
struct BsumShape {
    static constexpr bool ECH = PASS == 0 || PASS == 2;  // slabs over (n, chunk of e); else (n, chunk of m)
    static constexpr int RM = PASS == 1 ? VM : OM;       // rows of X
    static constexpr int CM = PASS == 0 ? OM : VM;       // rows of Y
    // slab length along k; with the padded row stride KP (odd, so that rows start in
    // different banks) both operands take 66-75 KB of LDS, so two workgroups fit a CU
    // (the complex64-integral forms are compiled for two waves per SIMD, the FP64 ones,
    // short of registers at that bound, for one)
    static constexpr int KM = PASS == 0 ? 128 : PASS == 1 ? 64 : 96;
    static constexpr int KP = KM + 1;
    static constexpr int PX = (RM * KM + 255) / 256, PY = (CM * KM + 255) / 256;
};

}  // namespace

template <int PASS, int OM, int VM, class IT>
__global__ __launch_bounds__(256, sizeof(IT) == 8 ? 2 : 1) void k_bsum_rb(SysDev s, const cd *t1, const cd *t2, cd *out) {
    using SH = BsumShape<PASS, OM, VM>;
    constexpr int KP = SH::KP, PX = SH::PX, PY = SH::PY;
    // integral operands are kept as stored until written to LDS
    using XT = std::conditional_t<PASS == 0 || PASS == 3, IT, cd>;
    using YT = std::conditional_t<PASS == 1 || PASS == 2, IT, cd>;
    __shared__ cd XS[SH::RM * KP], YS[SH::CM * KP];

    const int N = s.d.N, no = s.d.no, nv = s.d.nv;
    const int tid = threadIdx.x;
    const int R = PASS == 1 ? nv : no, C = PASS == 0 ? no : nv;
    const int R4 = (R + 3) & ~3, C4 = (C + 3) & ~3;
    const int lim = SH::ECH ? nv : no;            // range of the chunked index
    const int chunk = min(lim, SH::KM / nv);      // e (or m) values per slab
    const int K = chunk * nv;
    const int nslab = no * ((lim + chunk - 1) / chunk);
    const int nch = (lim + chunk - 1) / chunk;
    const int64_t n3 = (int64_t)N * N * N;
    const int64_t blk = blockIdx.x % n3;
    const int sp = (int)(blockIdx.x / n3), ns = fr_splits(s.d);
    const int r = (int)(blk % N), q = (int)((blk / N) % N), p = (int)(blk / ((int64_t)N * N));
    const int kb = kcv(s.kc, N, p, q, r);
    const int a0 = (int)((int64_t)sp * nslab / ns), a1 = (int)((int64_t)(sp + 1) * nslab / ns);
    const cd *tb = t2 + blk * s.d.t2blk();
    const IT *gb = nullptr;
    if constexpr (PASS == 0 || PASS == 1) gb = oovv_of<IT>(s) + blk * s.d.t2blk();
    if constexpr (PASS == 2) gb = ovvv_of<IT>(s) + blk3(N, q, p, r) * ((int64_t)no * nv * nv * nv);
    if constexpr (PASS == 3) gb = ooov_of<IT>(s) + blk * ((int64_t)no * no * no * nv);
    const FastDiv divK((uint32_t)K), divV((uint32_t)nv);
    const bool dress1 = (PASS == 0 || PASS == 1) && r == p, dress2 = (PASS == 0 || PASS == 1) && kb == p;

    // element offset of X(row, k) / Y(row, k) of slab (n, c0) with k = cq * nv + f
    auto xoff = [&](int row, int n, int c, int f) -> int64_t {
        if constexpr (PASS == 0) return (((int64_t)row * no + n) * nv + c) * nv + f;       // <m n||e f>, m = row
        if constexpr (PASS == 1) return (((int64_t)c * no + n) * nv + row) * nv + f;       // taut(m,n,a,f), a = row
        if constexpr (PASS == 2) return (((int64_t)row * no + n) * nv + c) * nv + f;       // t2(i,n,e,f), i = row
        return (((int64_t)c * no + n) * no + row) * nv + f;                                // <m n||i f>, i = row
    };
    auto yoff = [&](int row, int n, int c, int f) -> int64_t {
        if constexpr (PASS == 0) return (((int64_t)row * no + n) * nv + c) * nv + f;       // taut(i,n,e,f), i = row
        if constexpr (PASS == 1) return (((int64_t)c * no + n) * nv + row) * nv + f;       // <m n||e f>, e = row
        if constexpr (PASS == 2) return (((int64_t)n * nv + row) * nv + c) * nv + f;       // <n a||e f>, a = row
        return (((int64_t)c * no + n) * nv + row) * nv + f;                                // t2(m,n,a,f), a = row
    };
    // tau-tilde(x, n, y, f) - t2(x, n, y, f) on the blocks where t1 t1 enters
    auto dress = [&](int x, int n, int y, int f) -> cd {
        cd v = make_double2(0.0, 0.0);
        if (dress1) {
            const cd pp = cmul(t1[((int64_t)p * no + x) * nv + y], t1[((int64_t)q * no + n) * nv + f]);
            v.x += 0.5 * pp.x;
            v.y += 0.5 * pp.y;
        }
        if (dress2) {
            const cd pp = cmul(t1[((int64_t)p * no + x) * nv + f], t1[((int64_t)q * no + n) * nv + y]);
            v.x -= 0.5 * pp.x;
            v.y -= 0.5 * pp.y;
        }
        return v;
    };
    const XT *xsrc;
    const YT *ysrc;
    if constexpr (PASS == 0 || PASS == 3) xsrc = gb; else xsrc = tb;
    if constexpr (PASS == 1 || PASS == 2) ysrc = gb; else ysrc = tb;

    XT px[PX];
    YT py[PY];
    // staged element u of this thread: idx = tid + 256 u, row = idx / K, k = idx % K,
    // cq = k / nv, f = k % nv; addresses of absent elements are clamped to the slab start
#define BS_DECODE(idx, row, cq, f)               \
    const int row = (int)divK((uint32_t)(idx));  \
    const int k_ = (idx) - row * K;              \
    const int cq = (int)divV((uint32_t)k_);      \
    const int f = k_ - cq * nv;
#define BS_LOAD(it)                                                                          \
    {                                                                                        \
        const int n_ = (it) / nch, c0_ = ((it) % nch) * chunk;                               \
        _Pragma("unroll") for (int u = 0; u < PX; ++u) {                                     \
            const int idx = tid + 256 * u;                                                   \
            BS_DECODE(idx, row, cq, f)                                                       \
            const bool ok = idx < R4 * K && row < R && c0_ + cq < lim;                      \
            px[u] = xsrc[ok ? xoff(row, n_, c0_ + cq, f) : 0];                               \
        }                                                                                    \
        _Pragma("unroll") for (int u = 0; u < PY; ++u) {                                     \
            const int idx = tid + 256 * u;                                                   \
            BS_DECODE(idx, row, cq, f)                                                       \
            const bool ok = idx < C4 * K && row < C && c0_ + cq < lim;                      \
            py[u] = ysrc[ok ? yoff(row, n_, c0_ + cq, f) : 0];                               \
        }                                                                                    \
    }
#define BS_STORE(it)                                                                         \
    {                                                                                        \
        const int n_ = (it) / nch, c0_ = ((it) % nch) * chunk;                               \
        _Pragma("unroll") for (int u = 0; u < PX; ++u) {                                     \
            const int idx = tid + 256 * u;                                                   \
            BS_DECODE(idx, row, cq, f)                                                       \
            if (idx < R4 * K) {                                                              \
                const bool ok = row < R && c0_ + cq < lim;                                   \
                cd v = to_cd(px[u]);                                                         \
                if (PASS == 1 && ok && (dress1 || dress2)) v = cadd(v, dress(c0_ + cq, n_, row, f)); \
                XS[row * KP + k_] = ok ? v : make_double2(0.0, 0.0);                         \
            }                                                                                \
        }                                                                                    \
        _Pragma("unroll") for (int u = 0; u < PY; ++u) {                                     \
            const int idx = tid + 256 * u;                                                   \
            BS_DECODE(idx, row, cq, f)                                                       \
            if (idx < C4 * K) {                                                              \
                const bool ok = row < C && c0_ + cq < lim;                                   \
                cd v = to_cd(py[u]);                                                         \
                if (PASS == 0 && ok && (dress1 || dress2)) v = cadd(v, dress(row, n_, c0_ + cq, f)); \
                YS[row * KP + k_] = ok ? v : make_double2(0.0, 0.0);                         \
            }                                                                                \
        }                                                                                    \
    }

    // thread tiles over the actual rows and columns
    const int tr = R4 / 4, tc = C4 / 4, nt = tr * tc, ksn = 256 / nt;
    const int tile = tid / ksn, ks = tid % ksn;
    const bool act = tile < nt;
    const int r0 = act ? (tile / tc) * 4 : 0, c0 = act ? (tile % tc) * 4 : 0;
    cd acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = make_double2(0.0, 0.0);

    if (a0 < a1) {
        BS_LOAD(a0)
        BS_STORE(a0)
        __syncthreads();
        for (int it = a0; it < a1; ++it) {
            if (it + 1 < a1) BS_LOAD(it + 1)
            if (act) {
                for (int k = ks; k < K; k += ksn) {
                    cd x[4], y[4];
#pragma unroll
                    for (int d = 0; d < 4; ++d) {
                        x[d] = XS[(r0 + d) * KP + k];
                        y[d] = YS[(c0 + d) * KP + k];
                    }
#pragma unroll
                    for (int i = 0; i < 4; ++i)
#pragma unroll
                        for (int j = 0; j < 4; ++j) cfma(acc[i][j], x[i], y[j]);
                }
            }
            __syncthreads();
            if (it + 1 < a1) BS_STORE(it + 1)
            __syncthreads();
        }
    }
#undef BS_DECODE
#undef BS_LOAD
#undef BS_STORE

    // combine the ksn partial tiles in a fixed order, one tile row at a time (LDS reused)
    const double fac = PASS == 0 ? 0.5 : -0.5;
    cd *dst;
    int ld;
    if constexpr (PASS == 0) {
        dst = out + (sp * n3 + blk) * no * no;
        ld = no;
    } else if constexpr (PASS == 1) {
        dst = out + (sp * n3 + ((int64_t)r * N + p) * N + q) * nv * nv;
        ld = nv;
    } else if constexpr (PASS == 2) {
        dst = out + (sp * n3 + blk) * no * nv;
        ld = nv;
    } else {
        dst = out + (sp * n3 + ((int64_t)r * N + p) * N + q) * no * nv;
        ld = nv;
    }
    cd *red = XS;  // 1024 elements
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
        for (int j = 0; j < 4; ++j) red[tid * 4 + j] = acc[i][j];
        __syncthreads();
        if (tid < nt * 4) {
            const int tl = tid / 4, j = tid % 4;
            cd sum = make_double2(0.0, 0.0);
            for (int pp = 0; pp < ksn; ++pp) sum = cadd(sum, red[(tl * ksn + pp) * 4 + j]);
            const int row = (tl / tc) * 4 + i, col = (tl % tc) * 4 + j;
            if (row < R && col < C) dst[(int64_t)row * ld + col] = cscale(sum, fac);
        }
        __syncthreads();
    }
}

bool bsum_rb_fits(const Dims &d) { return d.no <= 16 && d.nv <= 32; }

template <int PASS, class IT>
static void launch_pass(const SysDev &s, const cd *t1, const cd *t2, cd *out, hipStream_t st) {
    const int64_t N = s.d.N;
    const dim3 grid((unsigned)(N * N * N * fr_splits(s.d)));
    hipLaunchKernelGGL((k_bsum_rb<PASS, 16, 32, IT>), grid, dim3(256), 0, st, s, t1, t2, out);
    CK_CHECK(hipGetLastError());
}

void launch_f_blocks_rb(const SysDev &s, const cd *t1, const cd *t2, cd *Poo, cd *Pvv, hipStream_t st) {
    if (s.oovv_c) {
        launch_pass<0, cf>(s, t1, t2, Poo, st);
        launch_pass<1, cf>(s, t1, t2, Pvv, st);
    } else {
        launch_pass<0, cd>(s, t1, t2, Poo, st);
        launch_pass<1, cd>(s, t1, t2, Pvv, st);
    }
}

void launch_r1_blocks_rb(const SysDev &s, const cd *t2, cd *P1a, cd *P1b, hipStream_t st) {
    if (s.ovvv_c) {
        launch_pass<2, cf>(s, nullptr, t2, P1a, st);
        launch_pass<3, cf>(s, nullptr, t2, P1b, st);
    } else {
        launch_pass<2, cd>(s, nullptr, t2, P1a, st);
        launch_pass<3, cd>(s, nullptr, t2, P1b, st);
    }
}

}  // namespace ck
