// Grouped complex FP64 GEMM over momentum-conserving blocks, on CDNA4 FP64 MFMA.
//
// Every contraction of the T2 residual that carries the N_band^6 N_k^4 cost (Sec. 3.1 of
// the paper; the eight-index sums of Sec. 4.3.4) becomes, once two momenta are fixed by
// a group label (total pair momentum K for the ladders, transfer q for the ring), a dense
// complex matrix product per group.  Operands are read in place from their canonical
// block layouts through per-row / per-column / per-k offset tables (GemmOps), so one
// kernel serves all five products without relayout passes; each table lookup is done
// once per tile row/column, and the k offsets of one tile are contiguous runs of at least
// n_vir (or n_occ^2) elements, so global loads stay coalesced.
//
// Tile: BM x BN complex outputs per 256-thread workgroup (4 waves as WM x WN), BK complex
// k-values per LDS stage, double buffered.  A complex multiply-accumulate is four real
// v_mfma_f64_16x16x4 products (re*re, -im*im into the real accumulator; re*im, im*re into
// the imaginary one).
#include "common.h"
#include "gemm_tiles.h"

namespace ck {

typedef double v4d __attribute__((ext_vector_type(4)));

template <int BM, int BN, int BK, int WM, int WN>
__global__ __launch_bounds__(256) void k_gemm_f64(GemmOps<cd> op) {
    constexpr int NT = 256;
    constexpr int TM = BM / WM, TN = BN / WN;
    constexpr int FM = TM / 16, FN = TN / 16;
    constexpr int RA = BM * BK / NT, RB = BN * BK / NT;  // complex loads per thread
    constexpr int ROWS_PER_PASS = NT / BK;
    static_assert(WM * WN == 4, "four waves");
    static_assert(BM * BK % NT == 0 && BN * BK % NT == 0, "tile/thread mismatch");

    __shared__ cd As[2][BK][BM + 1];
    __shared__ cd Bs[2][BK][BN + 1];

    const int tid = threadIdx.x;
    const int M = op.M, N = op.N, K = op.K;
    const GemmTile tile = gemm_tile((M + BM - 1) / BM, (N + BN - 1) / BN, op.G, 8);
    if (!tile.valid) return;
    const int g = tile.g;
    const int m0 = tile.mt * BM, n0 = tile.nt * BN;
    const int kl = tid % BK;        // this thread's k lane within a stage
    const int rl = tid / BK;        // first row/col handled by this thread

    // Per-thread row (A) and column (B) base offsets, clamped to a valid row; the loads are
    // branch free from always-valid addresses and out-of-range rows / k are zeroed when
    // the staged registers go to LDS, so loads stay in flight across the MFMA work.  The
    // k-table offsets are fetched one stage ahead of the data they address.
    int64_t arow[RA], bcol[RB];
    bool aok[RA], bok[RB];
#pragma unroll
    for (int i = 0; i < RA; ++i) {
        int m = m0 + rl + i * ROWS_PER_PASS;
        aok[i] = m < M;
        arow[i] = op.a_row[(int64_t)g * M + (aok[i] ? m : M - 1)];
    }
#pragma unroll
    for (int i = 0; i < RB; ++i) {
        int n = n0 + rl + i * ROWS_PER_PASS;
        bok[i] = n < N;
        bcol[i] = op.b_col[(int64_t)g * N + (bok[i] ? n : N - 1)];
    }

    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WN, wn = wave % WN;
    const int l16 = lane & 15, lk = lane >> 4;

    v4d acc_re[FM][FN], acc_im[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            acc_re[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
            acc_im[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
        }

    // Staged elements of the next stage and the k-table offsets of the one after it.
    // Every iteration loads (out-of-range elements read the zero buffer), so no
    // data-dependent select sits between a load and its LDS store.  Four rows per thread
    // (the 64 x 64 tile) in named registers; other tiles in component arrays (an array of
    // HIP vector structs would be kept in scratch memory).
    constexpr bool R4 = RA == 4 && RB == 4;
    cd ra0, ra1, ra2, ra3, rb0, rb1, rb2, rb3;
    double rax[RA], ray[RA], rbx[RB], rby[RB];
    int64_t ak_cur = 0, bk_cur = 0;
#define CK_KOFS(k0, ak, bk)                                \
    {                                                      \
        const int k_ = min((k0) + kl, K - 1);              \
        ak = op.a_k[(int64_t)g * K + k_];                  \
        bk = op.b_k[(int64_t)g * K + k_];                  \
    }
#define CK_LOAD(k0)                                                                                     \
    {                                                                                                   \
        const bool kin_ = (k0) + kl < K;                                                                \
        if constexpr (R4) {                                                                             \
            ra0 = *((kin_ && aok[0]) ? op.A + arow[0] + ak_cur : op.zeros);                             \
            ra1 = *((kin_ && aok[1]) ? op.A + arow[1] + ak_cur : op.zeros);                             \
            ra2 = *((kin_ && aok[2]) ? op.A + arow[2] + ak_cur : op.zeros);                             \
            ra3 = *((kin_ && aok[3]) ? op.A + arow[3] + ak_cur : op.zeros);                             \
            rb0 = *((kin_ && bok[0]) ? op.B + bcol[0] + bk_cur : op.zeros);                             \
            rb1 = *((kin_ && bok[1]) ? op.B + bcol[1] + bk_cur : op.zeros);                             \
            rb2 = *((kin_ && bok[2]) ? op.B + bcol[2] + bk_cur : op.zeros);                             \
            rb3 = *((kin_ && bok[3]) ? op.B + bcol[3] + bk_cur : op.zeros);                             \
        } else {                                                                                        \
            _Pragma("unroll") for (int i_ = 0; i_ < RA; ++i_) {                                         \
                const cd v_ = *((kin_ && aok[i_]) ? op.A + arow[i_] + ak_cur : op.zeros);               \
                rax[i_] = v_.x;                                                                         \
                ray[i_] = v_.y;                                                                         \
            }                                                                                           \
            _Pragma("unroll") for (int i_ = 0; i_ < RB; ++i_) {                                         \
                const cd v_ = *((kin_ && bok[i_]) ? op.B + bcol[i_] + bk_cur : op.zeros);               \
                rbx[i_] = v_.x;                                                                         \
                rby[i_] = v_.y;                                                                         \
            }                                                                                           \
        }                                                                                               \
    }
#define CK_STORE(buf)                                                                                  \
    {                                                                                                  \
        if constexpr (R4) {                                                                            \
            As[buf][kl][rl] = ra0;                                                                     \
            As[buf][kl][rl + ROWS_PER_PASS] = ra1;                                                     \
            As[buf][kl][rl + 2 * ROWS_PER_PASS] = ra2;                                                 \
            As[buf][kl][rl + 3 * ROWS_PER_PASS] = ra3;                                                 \
            Bs[buf][kl][rl] = rb0;                                                                     \
            Bs[buf][kl][rl + ROWS_PER_PASS] = rb1;                                                     \
            Bs[buf][kl][rl + 2 * ROWS_PER_PASS] = rb2;                                                 \
            Bs[buf][kl][rl + 3 * ROWS_PER_PASS] = rb3;                                                 \
        } else {                                                                                       \
            _Pragma("unroll") for (int i_ = 0; i_ < RA; ++i_)                                          \
                As[buf][kl][rl + i_ * ROWS_PER_PASS] = make_double2(rax[i_], ray[i_]);                 \
            _Pragma("unroll") for (int i_ = 0; i_ < RB; ++i_)                                          \
                Bs[buf][kl][rl + i_ * ROWS_PER_PASS] = make_double2(rbx[i_], rby[i_]);                 \
        }                                                                                              \
    }

    const int nk = (K + BK - 1) / BK;
    if (K > 0) {
        CK_KOFS(0, ak_cur, bk_cur);
        CK_LOAD(0);
        CK_STORE(0);
        CK_KOFS(BK, ak_cur, bk_cur);
    }
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        const int buf = kt & 1;
        int64_t ak_nxt, bk_nxt;
        CK_LOAD((kt + 1) * BK);  // zeros past the end
        CK_KOFS((kt + 2) * BK, ak_nxt, bk_nxt);
        // keep the prefetch issued here, ahead of the MFMA work it overlaps with
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            cd af[FM], bf[FN];
#pragma unroll
            for (int i = 0; i < FM; ++i) af[i] = As[buf][kk + lk][wm * TM + i * 16 + l16];
#pragma unroll
            for (int j = 0; j < FN; ++j) bf[j] = Bs[buf][kk + lk][wn * TN + j * 16 + l16];
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j) {
                    acc_re[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i].x, bf[j].x, acc_re[i][j], 0, 0, 0);
                    acc_re[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(-af[i].y, bf[j].y, acc_re[i][j], 0, 0, 0);
                    acc_im[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i].x, bf[j].y, acc_im[i][j], 0, 0, 0);
                    acc_im[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i].y, bf[j].x, acc_im[i][j], 0, 0, 0);
                }
        }
        __builtin_amdgcn_sched_barrier(0);
        CK_STORE(buf ^ 1);  // buf ^ 1 was last read before the previous barrier
        ak_cur = ak_nxt;
        bk_cur = bk_nxt;
        __syncthreads();
    }
#undef CK_KOFS
#undef CK_LOAD
#undef CK_STORE

    // epilogue: for the f64 16x16x4 MFMA, register r of a lane holds row 4*r + lane/16
    // of column lane%16 of each 16x16 tile
    const double alpha = op.alpha, beta = op.beta;
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            const int n = n0 + wn * TN + j * 16 + l16;
            if (n >= N) continue;
            const int64_t ccol = op.c_col[(int64_t)g * N + n];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + wm * TM + i * 16 + r * 4 + lk;
                if (m >= M) continue;
                cd *p = op.C + op.c_row[(int64_t)g * M + m] + ccol;
                cd v = make_double2(alpha * acc_re[i][j][r], alpha * acc_im[i][j][r]);
                if (beta != 0.0) {
                    cd o = *p;
                    v.x = fma(beta, o.x, v.x);
                    v.y = fma(beta, o.y, v.y);
                }
                *p = v;
            }
        }
}

// One thread per output element; for tests of the tiled kernel only.
__global__ void k_gemm_f64_reference(GemmOps<cd> op) {
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t total = (int64_t)op.G * op.M * op.N;
    if (idx >= total) return;
    int n = (int)(idx % op.N);
    int m = (int)((idx / op.N) % op.M);
    int g = (int)(idx / ((int64_t)op.N * op.M));
    cd acc = make_double2(0.0, 0.0);
    int64_t ar = op.a_row[(int64_t)g * op.M + m], bc = op.b_col[(int64_t)g * op.N + n];
    for (int k = 0; k < op.K; ++k)
        cfma(acc, op.A[ar + op.a_k[(int64_t)g * op.K + k]], op.B[bc + op.b_k[(int64_t)g * op.K + k]]);
    cd *p = op.C + op.c_row[(int64_t)g * op.M + m] + op.c_col[(int64_t)g * op.N + n];
    cd v = cscale(acc, op.alpha);
    if (op.beta != 0.0) v = cadd(v, cscale(*p, op.beta));
    *p = v;
}

template <int BM, int BN>
static void launch_f64(const GemmOps<cd> &op, hipStream_t s) {
    const dim3 grid = gemm_tile_grid((op.M + BM - 1) / BM, (op.N + BN - 1) / BN, op.G);
    hipLaunchKernelGGL((k_gemm_f64<BM, BN, 16, 2, 2>), grid, dim3(256), 0, s, op);
    CK_CHECK(hipGetLastError());
}

// Tile shapes of the FP64 product (gemm_tiles.h).  Every shape takes the same sixteen k
// per stage and the same order of MFMAs along k for each output element, so all of them
// give bitwise the same result; they differ in data reuse against the number of
// workgroups.
void gemm_f64_tile(const GemmOps<cd> &op, int tile, hipStream_t s) {
    if (op.G <= 0 || op.M <= 0 || op.N <= 0) return;
    switch (tile) {
        case F64_TILE_32x32: launch_f64<32, 32>(op, s); break;
        case F64_TILE_128x64: launch_f64<128, 64>(op, s); break;
        case F64_TILE_64x128: launch_f64<64, 128>(op, s); break;
        default: launch_f64<64, 64>(op, s); break;
    }
}

void gemm_f64(const GemmOps<cd> &op, hipStream_t s) { gemm_f64_tile(op, F64_TILE_64x64, s); }

void gemm_f64_reference(const GemmOps<cd> &op, hipStream_t s) {
    int64_t total = (int64_t)op.G * op.M * op.N;
    if (total <= 0) return;
    hipLaunchKernelGGL(k_gemm_f64_reference, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, op);
    CK_CHECK(hipGetLastError());
}

}  // namespace ck
